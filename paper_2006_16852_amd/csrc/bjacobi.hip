// bjacobi.hip -- block-Jacobi preconditioner (Sec. 3.2): batched
// Gauss-Jordan inversion of the diagonal blocks (one wave per block),
// adaptive storage precision of each inverse (binary16/32/64 chosen from
// the block's condition number and exponent range), the product z = M r,
// and the CG steps that use it (the r update fused with z = M r and the
// r.z, r.r reductions).
//
// Uniform blocks are consecutive ranges of BS rows (BS in {1,...,32}, the
// last one may be shorter), so a 256-row tile always holds whole blocks.
// Every inverse is stored as a BS x BS row-major array (zeros outside a
// short last block) at byte offset off[b] (a multiple of 16) in the
// precision prec[b].
//
// Variable-size blocks (at most 32 rows each, boundaries given or found by
// supervariable agglomeration) are inverted by the same elimination: blocks
// are sorted into classes by the power of two that holds them and each class
// runs the kernel of that width on a list of its blocks.  Block b's m x m
// inverse is stored row by row, each row padded to whole 16-byte chunks.
// A block reaches at most 31 rows beyond a 256-row tile, so the products
// stage the tile's vector part with 31 rows on either side in LDS.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "device_common.hpp"
#include "internal.hpp"

namespace mxl {

enum { BJ_P64 = 0, BJ_P32 = 1, BJ_P16 = 2 };

// Nearest-even rounding to binary16 from the format's definition: 11-bit
// significand, exponents -14..15, subnormal quantum 2^-24, overflow to
// infinity from 65520 on.  Scaling by the quantum is exact, rint rounds to
// nearest even.
__device__ __forceinline__ double round_f16(double x) {
    if (x == 0.0 || !__builtin_isfinite(x)) return x;
    const double a = fabs(x);
    if (a >= 65520.0) return copysign(__builtin_inf(), x);
    int e2;
    (void)frexp(a, &e2);
    int e = e2 - 1;
    if (e < -14) e = -14;
    const double quantum = ldexp(1.0, e - 10);
    return copysign(rint(a / quantum) * quantum, x);
}

// Lane l's value of v, as a wave-uniform scalar (l uniform).
__device__ __forceinline__ double lane_value(double v, int l) {
    const long long bits = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)bits, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One wave inverts one diagonal block (the 32-row shape, whose two
// register columns per lane leave no room for a second block).  Lane j holds column j of D and of
// its inverse I in registers (the block is staged through LDS once, row by
// row, to turn rows into columns); the pivot column's entries reach every
// lane as uniform scalars, so an elimination step is register arithmetic
// with no barrier.  Every element sees the same operations in the same
// order as a sequential Gauss-Jordan elimination with partial pivoting
// (first row of largest magnitude), with no multiply-add contraction, so
// the inverse, its condition number and the precision decision are
// reproducible.
// Rows of the block in slot `slot` of a launch: uniform blocks are slots
// themselves (b = slot, rows b*BS ..); with variable sizes the slot indexes
// a list of block ids of one size class and bptr gives the rows.
struct BlockSel {
    const int *list;      // variable sizes: block ids of this launch's class
    const int *bptr;      // variable sizes: block boundaries
    const int64_t *toff;  // variable sizes: offset of block b's m x m inverse in the output
};

template <int BS, bool VAR>
__device__ __forceinline__ void block_rows(int64_t slot, int64_t n, const BlockSel &sel, int64_t &b, int64_t &r0,
                                           int &m) {
    if constexpr (VAR) {
        b = sel.list[slot];
        r0 = sel.bptr[b];
        m = sel.bptr[b + 1] - (int)r0;
    } else {
        b = slot;
        r0 = b * BS;
        m = (int)(n - r0 < BS ? n - r0 : BS);
    }
}

// Row i of block b's inverse (lane j holds column j): uniform blocks are
// written BS x BS (zeros outside a short last block), variable ones m x m.
template <int BS, bool VAR>
__device__ __forceinline__ void store_inverse(double *__restrict__ inv, const BlockSel &sel, int64_t b, int m,
                                              int j, const double (&I)[BS], int p) {
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        double x = I[i];
        if (p == BJ_P32) x = (double)(float)x;
        else if (p == BJ_P16) x = round_f16(x);
        if constexpr (VAR) {
            if (i < m && j < m) inv[sel.toff[b] + (int64_t)i * m + j] = x;
        } else {
            inv[(b * BS + i) * BS + j] = x;
        }
    }
}

template <int BS, bool VAR>
__global__ __launch_bounds__(kWave) void k_bj_invert1(int64_t n, const int *__restrict__ rp,
                                                     const int *__restrict__ col,
                                                     const double *__restrict__ val, int adaptive,
                                                     double accuracy, double *__restrict__ inv,
                                                     double *__restrict__ cond, int *__restrict__ prec,
                                                     int *__restrict__ bad, BlockSel sel) {
#pragma clang fp contract(off)
    __shared__ double L[BS][BS + 1];
    int64_t b, r0;
    int m;
    block_rows<BS, VAR>(blockIdx.x, n, sel, b, r0, m);
    const int j = threadIdx.x;
    for (int e = j; e < BS * BS; e += kWave) L[e / BS][e % BS] = 0.0;
    __syncthreads();
    if (j < m)  // lane j loads row j of the block
        for (int k = rp[r0 + j]; k < rp[r0 + j + 1]; ++k) {
            const int64_t c = (int64_t)col[k] - r0;
            if (c >= 0 && c < m) L[j][c] = val[k];
        }
    __syncthreads();
    double D[BS], I[BS];
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        D[i] = j < BS ? L[i][j] : 0.0;
        I[i] = (i == j && j < m) ? 1.0 : 0.0;
    }
    auto norm1 = [&](const double (&M)[BS]) {
        double s = 0.0;
        if (j < m) {
#pragma unroll
            for (int i = 0; i < BS; ++i)
                if (i < m) s += fabs(M[i]);
        }
        return wave_max(s);
    };
    const double nD = norm1(D);
    bool singular = false;
#pragma clang loop unroll(full)
    for (int c = 0; c < BS; ++c) {
        if (singular || c >= m) continue;
        // pivot: the first row i >= c of largest |D[i][c]|, found by lane c
        double best = -1.0;
        int pv = c;
#pragma clang loop unroll(full)
        for (int i = c; i < BS; ++i)
            if (i < m) {
                const double a = fabs(D[i]);
                if (a > best) {
                    best = a;
                    pv = i;
                }
            }
        const double mx = lane_value(best, c);
        const int piv = __builtin_amdgcn_readlane(pv, c);
        if (!(mx > 0.0)) {  // singular block (zero column below the diagonal)
            singular = true;
            continue;
        }
        if (piv != c && j < m) {
            const double dc = D[c], ic = I[c];
#pragma clang loop unroll(full)
            for (int i = c + 1; i < BS; ++i)
                if (i == piv) {
                    D[c] = D[i];
                    I[c] = I[i];
                    D[i] = dc;
                    I[i] = ic;
                }
        }
        const double d = lane_value(D[c], c);
        if (j < m) {  // columns beyond a short last block stay zero
            D[c] = D[c] / d;
            I[c] = I[c] / d;
        }
#pragma clang loop unroll(full)
        for (int r = 0; r < BS; ++r) {
            if (r == c || r >= m) continue;
            const double f = lane_value(D[r], c);
            if (f == 0.0) continue;
            if (j < m) {
                const double pd = f * D[c];
                const double pi = f * I[c];
                D[r] = D[r] - pd;
                I[r] = I[r] - pi;
            }
        }
    }
    if (singular) {
        if (j == 0) atomicMin(bad, (int)(b < INT_MAX ? b : INT_MAX));
        return;
    }
    const double nI = norm1(I);
    const double kappa = nD * nI;
    int p = BJ_P64;
    if (adaptive) {
        double lo = __builtin_inf(), hi = 0.0;
        if (j < m) {
#pragma unroll
            for (int i = 0; i < BS; ++i) {
                if (i >= m) continue;
                const double a = fabs(I[i]);
                if (a == 0.0) continue;
                lo = a < lo ? a : lo;
                hi = a > hi ? a : hi;
            }
        }
        lo = -wave_max(-lo);
        hi = wave_max(hi);
        if (hi == 0.0) lo = hi = 1.0;
        if (kappa * ldexp(1.0, -11) <= accuracy && lo >= ldexp(1.0, -14) && hi <= 65504.0) p = BJ_P16;
        else if (kappa * ldexp(1.0, -24) <= accuracy && lo >= ldexp(1.0, -126) && hi <= 3.4028234663852886e38)
            p = BJ_P32;
    }
    if (j < BS) store_inverse<BS, VAR>(inv, sel, b, m, j, I, p);
    if (j == 0) {
        cond[b] = kappa;
        prec[b] = p;
    }
}

// Maximum over the BS lanes of a lane group (BS a power of two dividing
// the wave), with wave_max's comparison.
template <int BS, typename T>
__device__ __forceinline__ T group_max(T v) {
#pragma unroll
    for (int off = BS / 2; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// One wave inverts 64/BS diagonal blocks, one per group of BS lanes: lane
// j of a group holds column j of its block D and of the inverse I in
// registers (the blocks are staged through LDS once, row by row, to turn
// rows into columns; the loops over pivots and rows are unrolled).  Lane c
// of a group finds the pivot of column c and every entry of that column
// reaches the group's lanes by a lane shuffle, so an elimination step is
// register arithmetic with no barrier; a step that is zero in every block
// of the wave is skipped as a whole.  Every element sees the same
// operations in the same order as a sequential Gauss-Jordan elimination
// with partial pivoting (first row of largest magnitude), with no
// multiply-add contraction, so the inverse, its condition number and the
// precision decision are reproducible.
template <int BS, bool VAR>
__global__ __launch_bounds__(kWave) void k_bj_invert(int64_t n, const int *__restrict__ rp,
                                                     const int *__restrict__ col,
                                                     const double *__restrict__ val, int adaptive,
                                                     double accuracy, double *__restrict__ inv,
                                                     double *__restrict__ cond, int *__restrict__ prec,
                                                     int *__restrict__ bad, BlockSel sel, int64_t nslots) {
#pragma clang fp contract(off)
    constexpr int P = kWave / BS;
    __shared__ double L[P][BS][BS + 1];
    const int lane = threadIdx.x, q = lane / BS, j = lane % BS;
    const int src0 = q * BS;  // first lane of this lane's group
    const int64_t slot = (int64_t)blockIdx.x * P + q;
    const bool live = slot < nslots;
    int64_t b = 0, r0 = 0;
    int m = 0;
    if (live) block_rows<BS, VAR>(slot, n, sel, b, r0, m);
    for (int e = lane; e < P * BS * BS; e += kWave) L[e / (BS * BS)][(e / BS) % BS][e % BS] = 0.0;
    __syncthreads();
    if (j < m)  // lane j loads row j of its block
        for (int k = rp[r0 + j]; k < rp[r0 + j + 1]; ++k) {
            const int64_t c = (int64_t)col[k] - r0;
            if (c >= 0 && c < m) L[q][j][c] = val[k];
        }
    __syncthreads();
    double D[BS], I[BS];
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        D[i] = L[q][i][j];
        I[i] = (i == j && j < m) ? 1.0 : 0.0;
    }
    auto norm1 = [&](const double (&M)[BS]) {
        double s = 0.0;
        if (j < m) {
#pragma unroll
            for (int i = 0; i < BS; ++i)
                if (i < m) s += fabs(M[i]);
        }
        return group_max<BS>(s);
    };
    const double nD = norm1(D);
    bool singular = false;
#pragma clang loop unroll(full)
    for (int c = 0; c < BS; ++c) {
        // pivot: the first row i >= c of largest |D[i][c]|, found by lane c of the group
        double best = -1.0;
        int pv = c;
#pragma clang loop unroll(full)
        for (int i = c; i < BS; ++i)
            if (i < m) {
                const double a = fabs(D[i]);
                if (a > best) {
                    best = a;
                    pv = i;
                }
            }
        const double mx = __shfl(best, src0 + c, kWave);
        const int piv = __shfl(pv, src0 + c, kWave);
        bool act = !singular && c < m;
        if (act && !(mx > 0.0)) {  // singular block (zero column below the diagonal)
            singular = true;
            act = false;
        }
        if (act && piv != c && j < m) {
            const double dc = D[c], ic = I[c];
#pragma clang loop unroll(full)
            for (int i = c + 1; i < BS; ++i)
                if (i == piv) {
                    D[c] = D[i];
                    I[c] = I[i];
                    D[i] = dc;
                    I[i] = ic;
                }
        }
        const double d = __shfl(D[c], src0 + c, kWave);
        if (act && j < m) {  // columns beyond a short last block stay zero
            D[c] = D[c] / d;
            I[c] = I[c] / d;
        }
#pragma clang loop unroll(full)
        for (int r = 0; r < BS; ++r) {
            if (r == c) continue;
            const double f = __shfl(D[r], src0 + c, kWave);
            const bool upd = act && r < m && f != 0.0;
            if (!__any(upd)) continue;
            if (upd && j < m) {
                const double pd = f * D[c];
                const double pi = f * I[c];
                D[r] = D[r] - pd;
                I[r] = I[r] - pi;
            }
        }
    }
    if (singular && j == 0) atomicMin(bad, (int)(b < INT_MAX ? b : INT_MAX));
    const double nI = norm1(I);
    const double kappa = nD * nI;
    int p = BJ_P64;
    if (adaptive) {
        double lo = __builtin_inf(), hi = 0.0;
        if (j < m) {
#pragma unroll
            for (int i = 0; i < BS; ++i) {
                if (i >= m) continue;
                const double a = fabs(I[i]);
                if (a == 0.0) continue;
                lo = a < lo ? a : lo;
                hi = a > hi ? a : hi;
            }
        }
        lo = -group_max<BS>(-lo);
        hi = group_max<BS>(hi);
        if (hi == 0.0) lo = hi = 1.0;
        if (kappa * ldexp(1.0, -11) <= accuracy && lo >= ldexp(1.0, -14) && hi <= 65504.0) p = BJ_P16;
        else if (kappa * ldexp(1.0, -24) <= accuracy && lo >= ldexp(1.0, -126) && hi <= 3.4028234663852886e38)
            p = BJ_P32;
    }
    if (live && !singular) {
        store_inverse<BS, VAR>(inv, sel, b, m, j, I, p);
        if (j == 0) {
            cond[b] = kappa;
            prec[b] = p;
        }
    }
}

// Packs the rounded inverses into their storage precision (the values are
// already representable, so the conversions are exact).
template <int BS>
__global__ void k_bj_pack(int64_t nb, const double *__restrict__ inv, const int *__restrict__ prec,
                          const int64_t *__restrict__ off, unsigned char *__restrict__ store) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nb * BS * BS) return;
    const int64_t b = e / (BS * BS), k = e % (BS * BS);
    unsigned char *base = store + off[b];
    const double x = inv[e];
    switch (prec[b]) {
    case BJ_P16: ((_Float16 *)base)[k] = (_Float16)x; break;
    case BJ_P32: ((float *)base)[k] = (float)x; break;
    default: ((double *)base)[k] = x; break;
    }
}

// Row t of block b's stored inverse times the block's vector part held in
// LDS (xs[0..BS)), summed over ascending columns in FP64.  Blocks start at
// 16-byte-aligned offsets, so a row whose bytes are a multiple of 16 is
// read with 16-byte vector loads (8 binary16, 4 binary32 or 2 binary64
// values each); other rows element by element.
template <typename T, int BS>
__device__ __forceinline__ double bj_row_t(const unsigned char *__restrict__ base, int t, const double *xs) {
    constexpr int E = 16 / (int)sizeof(T);
    double s = 0.0;
    if constexpr (BS * sizeof(T) % 16 == 0) {
        typedef T TV __attribute__((ext_vector_type(E)));
        const TV *rp = (const TV *)base + t * (BS / E);
#pragma unroll
        for (int c = 0; c < BS / E; ++c) {
            const TV v = rp[c];
#pragma unroll
            for (int e = 0; e < E; ++e) s += (double)v[e] * xs[c * E + e];
        }
    } else {
        const T *rp = (const T *)base + t * BS;
#pragma unroll
        for (int j = 0; j < BS; ++j) s += (double)rp[j] * xs[j];
    }
    return s;
}

template <int BS>
__device__ __forceinline__ double bj_row(const unsigned char *__restrict__ store, int64_t off, int pr,
                                         int t, const double *xs) {
    const unsigned char *base = store + off;
    if (pr == BJ_P16) return bj_row_t<_Float16, BS>(base, t, xs);
    if (pr == BJ_P32) return bj_row_t<float, BS>(base, t, xs);
    return bj_row_t<double, BS>(base, t, xs);
}

// z = M r on 256-row tiles (whole blocks): each wave parks its 64 values of
// r in LDS, then lane l forms row (l mod BS) of its block.
#define MXL_BJ_TILE(n)                                                  \
    const int L = blockIdx.x;                                           \
    int64_t tb_, te_;                                                   \
    int ts_;                                                            \
    band_walk(((n) + kWG - 1) / kWG, blockIdx.x, gridDim.x, tb_, te_, ts_);

template <int BS>
__global__ __launch_bounds__(kWG) void k_bj_apply(int64_t n, const unsigned char *__restrict__ store,
                                                  const int64_t *__restrict__ off,
                                                  const int *__restrict__ prec, double alpha,
                                                  const double *__restrict__ r, double beta,
                                                  double *__restrict__ z, const int *stop) {
    if (stop && *stop) return;  // inside a solve: nothing after a device-side stop uses z
    __shared__ double xs[kWG];
    MXL_BJ_TILE(n)
    (void)L;
    const int lane = threadIdx.x;
    for (int64_t t_ = tb_; t_ < te_; t_ += ts_) {
        const int64_t i = t_ * kWG + lane;
        xs[lane] = i < n ? r[i] : 0.0;
        __syncthreads();
        if (i < n) {
            const int64_t blk = i / BS;
            const int t = (int)(i % BS);
            const double v = bj_row<BS>(store, off[blk], prec[blk], t, xs + (lane - t));
            z[i] = beta == 0.0 ? alpha * v : alpha * v + beta * z[i];
        }
        __syncthreads();
    }
}

// CG with block Jacobi, initial step: z = M r, p = z; publishes [r.z, r.r, b.b].
// V is the vector type: with binary32 vectors z is rounded to binary32
// before it enters p and r.z (the inverses are still applied in FP64).
template <typename V, int BS>
__global__ __launch_bounds__(kWG) void k_cg_init_bj(int64_t n, const V *__restrict__ b,
                                                    const V *__restrict__ r, V *__restrict__ p,
                                                    const unsigned char *__restrict__ store,
                                                    const int64_t *__restrict__ off,
                                                    const int *__restrict__ prec,
                                                    double *__restrict__ parts) {
    __shared__ double xs[kWG];
    MXL_BJ_TILE(n)
    const int lane = threadIdx.x;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int64_t t_ = tb_; t_ < te_; t_ += ts_) {
        const int64_t i = t_ * kWG + lane;
        const double ri = i < n ? (double)r[i] : 0.0;
        xs[lane] = ri;
        __syncthreads();
        if (i < n) {
            const int64_t blk = i / BS;
            const int t = (int)(i % BS);
            const V zv = (V)bj_row<BS>(store, off[blk], prec[blk], t, xs + (lane - t));
            p[i] = zv;
            rz += ri * (double)zv;
            rr += ri * ri;
            bb += (double)b[i] * (double)b[i];
        }
        __syncthreads();
    }
    double v[3] = {rz, rr, bb};
    publish<3>(v, parts, L);
}

// CG with block Jacobi, after the fused p.q: alpha = rho_{k-1} / p.q,
// r -= alpha q (in FP64, rounded to V), z = M r (rounded to V), and the
// reductions r.z, r.r.  The stop handshake with k_cg_pupdate (st->ustop) is
// the one of the point-Jacobi kernels.
template <typename V, int BS>
__global__ __launch_bounds__(kWG) void k_cg_update_bj(int64_t n, V *__restrict__ r,
                                                      const V *__restrict__ q, V *__restrict__ z,
                                                      const unsigned char *__restrict__ store,
                                                      const int64_t *__restrict__ off,
                                                      const int *__restrict__ prec, SolverState *st,
                                                      const double *__restrict__ pq_parts, int pq_slots,
                                                      double *__restrict__ parts, int k) {
    __shared__ double xs[kWG];
    if (st->stop) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->ustop = 1;
        return;
    }
    double eta[1];
    gather_all<1>(pq_parts, pq_slots, eta);
    const bool chk = st->nonfinite_check != 0;
    const bool nonfin = chk && !finite_d(eta[0]);
    if (nonfin || eta[0] <= 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->stop = nonfin ? ST_NONFINITE : ST_BREAKDOWN;
            st->ustop = 1;
            st->iters = k - 1;
            st->eta = eta[0];
        }
        return;
    }
    const double alpha = st->rho2[(k - 1) & 1] / eta[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->alpha = alpha;
        st->eta = eta[0];
        st->ustop = 0;
    }
    MXL_BJ_TILE(n)
    const int lane = threadIdx.x;
    double rz = 0.0, rr = 0.0;
    for (int64_t t_ = tb_; t_ < te_; t_ += ts_) {
        const int64_t i = t_ * kWG + lane;
        double ri = 0.0;
        if (i < n) {
            V rv;
            if constexpr (sizeof(V) == 8) rv = r[i] - alpha * q[i];
            else rv = (V)((double)r[i] - alpha * (double)q[i]);
            r[i] = rv;
            ri = (double)rv;
        }
        xs[lane] = ri;
        __syncthreads();
        if (i < n) {
            const int64_t blk = i / BS;
            const int t = (int)(i % BS);
            const V zv = (V)bj_row<BS>(store, off[blk], prec[blk], t, xs + (lane - t));
            z[i] = zv;
            rz += ri * (double)zv;
            rr += ri * ri;
        }
        __syncthreads();
    }
    double v[2] = {rz, rr};
    publish<2>(v, parts, L);
}

// ------------------------------------------------ variable-size blocks
constexpr int kBjMax = 32;            // largest block
constexpr int kBjHalo = kBjMax - 1;   // rows a block can reach beyond a tile
constexpr int kBjWin = kWG + 2 * kBjHalo;

// same[i] = 1 when row i has exactly the column set of row i - 1 (a
// supervariable continues), 0 otherwise (same[0] = 0).
__global__ void k_bj_same_prev(int64_t n, const int *__restrict__ rp, const int *__restrict__ col,
                               unsigned char *__restrict__ same) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned char f = 0;
    if (i > 0) {
        const int a0 = rp[i - 1], a1 = rp[i], b1 = rp[i + 1];
        if (a1 - a0 == b1 - a1) {
            f = 1;
            for (int k = 0; k < a1 - a0; ++k)
                if (col[a0 + k] != col[a1 + k]) {
                    f = 0;
                    break;
                }
        }
    }
    same[i] = f;
}

// rblk[i] = b for every row of block b (one thread per block).
__global__ void k_bj_rowmap(int64_t nb, const int *__restrict__ bptr, int *__restrict__ rblk) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    for (int i = bptr[b]; i < bptr[b + 1]; ++i) rblk[i] = (int)b;
}

// 16-byte chunks per stored row of an m-wide block in precision pr.
__host__ __device__ __forceinline__ int bjv_chunks(int m, int pr) {
    const int e = pr == BJ_P16 ? 8 : pr == BJ_P32 ? 4 : 2;
    return (m + e - 1) / e;
}

// Packs block b's m x m inverse (FP64, already rounded to its precision)
// into rows of whole 16-byte chunks, padding with zeros; one workgroup per
// block.
__global__ void k_bj_pack_var(int64_t nb, const int *__restrict__ bptr, const int64_t *__restrict__ toff,
                              const double *__restrict__ inv, const int *__restrict__ prec,
                              const int64_t *__restrict__ off, unsigned char *__restrict__ store) {
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    const int m = bptr[b + 1] - bptr[b], pr = prec[b];
    const int ld = bjv_chunks(m, pr) * (pr == BJ_P16 ? 8 : pr == BJ_P32 ? 4 : 2);
    unsigned char *base = store + off[b];
    for (int e = threadIdx.x; e < m * ld; e += blockDim.x) {
        const int i = e / ld, j = e % ld;
        const double x = j < m ? inv[toff[b] + (int64_t)i * m + j] : 0.0;
        switch (pr) {
        case BJ_P16: ((_Float16 *)base)[e] = (_Float16)x; break;
        case BJ_P32: ((float *)base)[e] = (float)x; break;
        default: ((double *)base)[e] = x; break;
        }
    }
}

// Row t of an m-wide stored inverse times xs[0..m), ascending columns, FP64;
// 16-byte loads, the padding lanes of the last chunk are not multiplied (a
// neighbouring row's Inf or NaN must not reach this row).
template <typename T>
__device__ __forceinline__ double bjv_row_t(const unsigned char *__restrict__ base, int t, int m,
                                            const double *xs) {
    constexpr int E = 16 / (int)sizeof(T);
    typedef T TV __attribute__((ext_vector_type(E)));
    const int nv = (m + E - 1) / E;
    const TV *rowp = (const TV *)base + (int64_t)t * nv;
    double s = 0.0;
    for (int c = 0; c < nv; ++c) {
        const TV v = rowp[c];
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (c * E + e < m) s += (double)v[e] * xs[c * E + e];
    }
    return s;
}

__device__ __forceinline__ double bjv_row(const unsigned char *__restrict__ store, int64_t off, int pr, int t,
                                          int m, const double *xs) {
    const unsigned char *base = store + off;
    if (pr == BJ_P16) return bjv_row_t<_Float16>(base, t, m, xs);
    if (pr == BJ_P32) return bjv_row_t<float>(base, t, m, xs);
    return bjv_row_t<double>(base, t, m, xs);
}

// Block row of row i (inside the tile starting at t0) against the staged
// window xw = rows t0 - kBjHalo .. t0 + kWG + kBjHalo.
__device__ __forceinline__ double bjv_apply_row(int64_t i, int64_t t0, const int *__restrict__ rblk,
                                                const int *__restrict__ bptr,
                                                const unsigned char *__restrict__ store,
                                                const int64_t *__restrict__ off, const int *__restrict__ prec,
                                                const double *xw) {
    const int b = rblk[i];
    const int r0 = bptr[b], m = bptr[b + 1] - r0;
    return bjv_row(store, off[b], prec[b], (int)(i - r0), m, xw + (r0 - (t0 - kBjHalo)));
}

// z = alpha M r + beta z with variable-size blocks.
__global__ __launch_bounds__(kWG) void k_bj_apply_var(int64_t n, const int *__restrict__ rblk,
                                                      const int *__restrict__ bptr,
                                                      const unsigned char *__restrict__ store,
                                                      const int64_t *__restrict__ off,
                                                      const int *__restrict__ prec, double alpha,
                                                      const double *__restrict__ r, double beta,
                                                      double *__restrict__ z, const int *stop) {
    if (stop && *stop) return;
    __shared__ double xw[kBjWin];
    MXL_BJ_TILE(n)
    (void)L;
    const int lane = threadIdx.x;
    for (int64_t t_ = tb_; t_ < te_; t_ += ts_) {
        const int64_t t0 = t_ * kWG;
        for (int w = lane; w < kBjWin; w += kWG) {
            const int64_t row = t0 - kBjHalo + w;
            xw[w] = row >= 0 && row < n ? r[row] : 0.0;
        }
        __syncthreads();
        const int64_t i = t0 + lane;
        if (i < n) {
            const double v = bjv_apply_row(i, t0, rblk, bptr, store, off, prec, xw);
            z[i] = beta == 0.0 ? alpha * v : alpha * v + beta * z[i];
        }
        __syncthreads();
    }
}

// CG initial step with variable-size blocks: z = M r, p = z; publishes
// [r.z, r.r, b.b] (as k_cg_init_bj).
template <typename V>
__global__ __launch_bounds__(kWG) void k_cg_init_bjv(int64_t n, const V *__restrict__ b,
                                                     const V *__restrict__ r, V *__restrict__ p,
                                                     const int *__restrict__ rblk, const int *__restrict__ bptr,
                                                     const unsigned char *__restrict__ store,
                                                     const int64_t *__restrict__ off,
                                                     const int *__restrict__ prec, double *__restrict__ parts) {
    __shared__ double xw[kBjWin];
    MXL_BJ_TILE(n)
    const int lane = threadIdx.x;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int64_t t_ = tb_; t_ < te_; t_ += ts_) {
        const int64_t t0 = t_ * kWG;
        for (int w = lane; w < kBjWin; w += kWG) {
            const int64_t row = t0 - kBjHalo + w;
            xw[w] = row >= 0 && row < n ? (double)r[row] : 0.0;
        }
        __syncthreads();
        const int64_t i = t0 + lane;
        if (i < n) {
            const double ri = xw[lane + kBjHalo];
            const V zv = (V)bjv_apply_row(i, t0, rblk, bptr, store, off, prec, xw);
            p[i] = zv;
            rz += ri * (double)zv;
            rr += ri * ri;
            bb += (double)b[i] * (double)b[i];
        }
        __syncthreads();
    }
    double v[3] = {rz, rr, bb};
    publish<3>(v, parts, L);
}

// CG update with variable-size blocks: as k_cg_update_bj, but r_out =
// r_in - alpha q goes to a second buffer, because each workgroup also forms
// the new residual of the 31 rows on either side of its tile (the rows its
// blocks reach into) from r_in, which its neighbours must not overwrite.
template <typename V>
__global__ __launch_bounds__(kWG) void k_cg_update_bjv(int64_t n, const V *__restrict__ r_in,
                                                       V *__restrict__ r_out, const V *__restrict__ q,
                                                       V *__restrict__ z, const int *__restrict__ rblk,
                                                       const int *__restrict__ bptr,
                                                       const unsigned char *__restrict__ store,
                                                       const int64_t *__restrict__ off,
                                                       const int *__restrict__ prec, SolverState *st,
                                                       const double *__restrict__ pq_parts, int pq_slots,
                                                       double *__restrict__ parts, int k) {
    __shared__ double xw[kBjWin];
    if (st->stop) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->ustop = 1;
        return;
    }
    double eta[1];
    gather_all<1>(pq_parts, pq_slots, eta);
    const bool chk = st->nonfinite_check != 0;
    const bool nonfin = chk && !finite_d(eta[0]);
    if (nonfin || eta[0] <= 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->stop = nonfin ? ST_NONFINITE : ST_BREAKDOWN;
            st->ustop = 1;
            st->iters = k - 1;
            st->eta = eta[0];
        }
        return;
    }
    const double alpha = st->rho2[(k - 1) & 1] / eta[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->alpha = alpha;
        st->eta = eta[0];
        st->ustop = 0;
    }
    MXL_BJ_TILE(n)
    const int lane = threadIdx.x;
    double rz = 0.0, rr = 0.0;
    for (int64_t t_ = tb_; t_ < te_; t_ += ts_) {
        const int64_t t0 = t_ * kWG;
        for (int w = lane; w < kBjWin; w += kWG) {
            const int64_t row = t0 - kBjHalo + w;
            double rv = 0.0;
            if (row >= 0 && row < n) {
                V v;
                if constexpr (sizeof(V) == 8) v = r_in[row] - alpha * q[row];
                else v = (V)((double)r_in[row] - alpha * (double)q[row]);
                rv = (double)v;
                if (w >= kBjHalo && w < kBjHalo + kWG) r_out[row] = v;
            }
            xw[w] = rv;
        }
        __syncthreads();
        const int64_t i = t0 + lane;
        if (i < n) {
            const double ri = xw[lane + kBjHalo];
            const V zv = (V)bjv_apply_row(i, t0, rblk, bptr, store, off, prec, xw);
            z[i] = zv;
            rz += ri * (double)zv;
            rr += ri * ri;
        }
        __syncthreads();
    }
    double v[2] = {rz, rr};
    publish<2>(v, parts, L);
}

// ------------------------------------------------------------ host side
#define MXL_BS_SWITCH(BSV, ...)                      \
    switch (BSV) {                                   \
    case 1: { constexpr int BS = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int BS = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int BS = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int BS = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int BS = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int BS = 32; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;            \
    }

hipError_t bj_cg_init(const mxl_ctx *ctx, const JacobiImpl &P, int dtype, int64_t n, const void *b,
                      const void *r, void *p, double *parts, hipStream_t s) {
    const int g = vec_grid(ctx, n);
    const unsigned char *store = (const unsigned char *)P.bstore->p;
    const int64_t *off = (const int64_t *)P.boff->p;
    const int *prec = (const int *)P.bprec->p;
    if (P.var) {
        const int *rb = (const int *)P.rblk->p, *bp = (const int *)P.bptr_d->p;
        if (dtype == MXL_F32)
            hipLaunchKernelGGL(k_cg_init_bjv<float>, dim3(g), dim3(kWG), 0, s, n, (const float *)b,
                               (const float *)r, (float *)p, rb, bp, store, off, prec, parts);
        else
            hipLaunchKernelGGL(k_cg_init_bjv<double>, dim3(g), dim3(kWG), 0, s, n, (const double *)b,
                               (const double *)r, (double *)p, rb, bp, store, off, prec, parts);
        return hipGetLastError();
    }
    if (dtype == MXL_F32) {
        MXL_BS_SWITCH(P.bs, hipLaunchKernelGGL((k_cg_init_bj<float, BS>), dim3(g), dim3(kWG), 0, s, n,
                                               (const float *)b, (const float *)r, (float *)p, store, off,
                                               prec, parts));
    } else {
        MXL_BS_SWITCH(P.bs, hipLaunchKernelGGL((k_cg_init_bj<double, BS>), dim3(g), dim3(kWG), 0, s, n,
                                               (const double *)b, (const double *)r, (double *)p, store, off,
                                               prec, parts));
    }
    return hipGetLastError();
}

hipError_t bj_cg_update(const mxl_ctx *ctx, const JacobiImpl &P, int dtype, int64_t n, const void *r_in,
                        void *r_out, const void *q, void *z, SolverState *st, const double *pq_parts, int pq_slots,
                        double *parts, int k, hipStream_t s) {
    const int g = vec_grid(ctx, n);
    const unsigned char *store = (const unsigned char *)P.bstore->p;
    const int64_t *off = (const int64_t *)P.boff->p;
    const int *prec = (const int *)P.bprec->p;
    if (P.var) {
        if (r_in == r_out) return hipErrorInvalidValue;
        const int *rb = (const int *)P.rblk->p, *bp = (const int *)P.bptr_d->p;
        if (dtype == MXL_F32)
            hipLaunchKernelGGL(k_cg_update_bjv<float>, dim3(g), dim3(kWG), 0, s, n, (const float *)r_in,
                               (float *)r_out, (const float *)q, (float *)z, rb, bp, store, off, prec, st, pq_parts,
                               pq_slots, parts, k);
        else
            hipLaunchKernelGGL(k_cg_update_bjv<double>, dim3(g), dim3(kWG), 0, s, n, (const double *)r_in,
                               (double *)r_out, (const double *)q, (double *)z, rb, bp, store, off, prec, st,
                               pq_parts, pq_slots, parts, k);
        return hipGetLastError();
    }
    if (r_in != r_out) return hipErrorInvalidValue;
    void *r = r_out;
    if (dtype == MXL_F32) {
        MXL_BS_SWITCH(P.bs, hipLaunchKernelGGL((k_cg_update_bj<float, BS>), dim3(g), dim3(kWG), 0, s, n,
                                               (float *)r, (const float *)q, (float *)z, store, off, prec, st,
                                               pq_parts, pq_slots, parts, k));
    } else {
        MXL_BS_SWITCH(P.bs, hipLaunchKernelGGL((k_cg_update_bj<double, BS>), dim3(g), dim3(kWG), 0, s, n,
                                               (double *)r, (const double *)q, (double *)z, store, off, prec,
                                               st, pq_parts, pq_slots, parts, k));
    }
    return hipGetLastError();
}

hipError_t bj_apply(const mxl_ctx *ctx, const JacobiImpl &P, int64_t n, double alpha, const void *r,
                    double beta, void *z, hipStream_t s, const int *stop) {
    const int g = vec_grid(ctx, n);
    if (P.var) {
        hipLaunchKernelGGL(k_bj_apply_var, dim3(g), dim3(kWG), 0, s, n, (const int *)P.rblk->p,
                           (const int *)P.bptr_d->p, (const unsigned char *)P.bstore->p, (const int64_t *)P.boff->p,
                           (const int *)P.bprec->p, alpha, (const double *)r, beta, (double *)z, stop);
        return hipGetLastError();
    }
    MXL_BS_SWITCH(P.bs, hipLaunchKernelGGL(k_bj_apply<BS>, dim3(g), dim3(kWG), 0, s, n,
                                           (const unsigned char *)P.bstore->p, (const int64_t *)P.boff->p,
                                           (const int *)P.bprec->p, alpha, (const double *)r, beta,
                                           (double *)z, stop));
    return hipGetLastError();
}

static hipError_t bj_invert(const MatrixImpl &A, int bs, int adaptive, double accuracy, double *inv,
                            double *cond, int *prec, int *bad, hipStream_t s) {
    const int64_t nb = (A.nrows + bs - 1) / bs;
    const BlockSel none{nullptr, nullptr, nullptr};
    if (bs == 32)
        hipLaunchKernelGGL((k_bj_invert1<32, false>), dim3((unsigned)nb), dim3(kWave), 0, s, A.nrows,
                           (const int *)A.row_ptr->p, (const int *)A.col->p, (const double *)A.val->p, adaptive,
                           accuracy, inv, cond, prec, bad, none);
    else {
#define MXL_BJ_INV(BSV)                                                                                     \
    case BSV:                                                                                               \
        hipLaunchKernelGGL((k_bj_invert<BSV, false>), dim3((unsigned)((nb + kWave / BSV - 1) / (kWave / BSV))), \
                           dim3(kWave), 0, s, A.nrows, (const int *)A.row_ptr->p, (const int *)A.col->p,     \
                           (const double *)A.val->p, adaptive, accuracy, inv, cond, prec, bad, none, nb);   \
        break;
        switch (bs) {
            MXL_BJ_INV(1) MXL_BJ_INV(2) MXL_BJ_INV(4) MXL_BJ_INV(8) MXL_BJ_INV(16)
        default: return hipErrorInvalidValue;
        }
#undef MXL_BJ_INV
    }
    return hipGetLastError();
}

static hipError_t bj_pack(int bs, int64_t nb, const double *inv, const int *prec, const int64_t *off,
                          unsigned char *store, hipStream_t s) {
    const int64_t total = nb * bs * bs;
    const unsigned g = (unsigned)((total + 255) / 256);
    MXL_BS_SWITCH(bs, hipLaunchKernelGGL(k_bj_pack<BS>, dim3(g), dim3(256), 0, s, nb, inv, prec, off, store));
    return hipGetLastError();
}

}  // namespace mxl

using namespace mxl;

extern "C" mxl_status mxl_bjacobi_generate(const mxl_op *Aop, int32_t block_size, int32_t adaptive,
                                           double accuracy, mxl_op **Pout) try {
    if (!Aop || !Pout || Aop->kind != MXL_OP_MATRIX)
        return set_error(MXL_ERR_INVALID_ARG, "matrix operator and output required");
    *Pout = nullptr;
    const auto &A = Aop->mat;
    if (block_size != 1 && block_size != 2 && block_size != 4 && block_size != 8 && block_size != 16 &&
        block_size != 32)
        return set_error(MXL_ERR_INVALID_ARG, "block_size must be 1, 2, 4, 8, 16 or 32");
    if (A->nrows != A->ncols) return set_error(MXL_ERR_NOT_IMPLEMENTED, "block Jacobi needs a square matrix");
    if (A->dtype != MXL_F64) return set_error(MXL_ERR_NOT_IMPLEMENTED, "block Jacobi needs an FP64 matrix");
    if (A->format == MXL_FMT_STENCIL)
        return set_error(MXL_ERR_NOT_IMPLEMENTED, "block Jacobi needs stored matrix rows");
    if (A->nrows == 0) return set_error(MXL_ERR_INVALID_ARG, "empty matrix");
    if (!(accuracy >= 0.0)) return set_error(MXL_ERR_INVALID_ARG, "accuracy must be >= 0");
    if (accuracy == 0.0) accuracy = 0.1;
    DeviceScope ds(A->ctx->device);
    hipStream_t s = A->ctx->stream;
    const int bs = block_size;
    const int64_t nb = (A->nrows + bs - 1) / bs;
    auto J = std::make_shared<JacobiImpl>();
    J->A = A;
    J->block = true;
    J->bs = bs;
    J->nblocks = nb;
    hipError_t e = hipSuccess;
    BufPtr tmp, bad;
    auto mk = [&](size_t bytes) {
        auto d = std::make_shared<DevBuf>();
        if (hipMalloc(&d->p, bytes ? bytes : 16) != hipSuccess) return BufPtr();
        d->bytes = bytes;
        d->owned = true;
        return d;
    };
    tmp = mk((size_t)nb * bs * bs * 8);
    J->bcond = mk((size_t)nb * 8);
    J->bprec = mk((size_t)nb * 4);
    J->boff = mk((size_t)nb * 8);
    bad = mk(4);
    if (!tmp || !J->bcond || !J->bprec || !J->boff || !bad)
        return set_error(MXL_ERR_OUT_OF_MEMORY, "block Jacobi workspace");
    int none = INT_MAX;
    if ((e = hipMemcpyAsync(bad->p, &none, 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = bj_invert(*A, bs, adaptive ? 1 : 0, accuracy, (double *)tmp->p, (double *)J->bcond->p,
                       (int *)J->bprec->p, (int *)bad->p, s)) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, std::string("block inversion: ") + hipGetErrorString(e));
    int hb = INT_MAX;
    std::vector<int> hp((size_t)nb);
    if (hipMemcpyAsync(&hb, bad->p, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hp.data(), J->bprec->p, (size_t)nb * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "block inversion read-back");
    if (hb != INT_MAX) {
        char msg[96];
        snprintf(msg, sizeof msg, "diagonal block %d is singular", hb);
        return set_error(MXL_ERR_ZERO_DIAG, msg);
    }
    // byte offsets: each block padded to a multiple of 16 bytes (vector row loads)
    std::vector<int64_t> ho((size_t)nb);
    int64_t total = 0;
    for (int64_t b = 0; b < nb; ++b) {
        ho[b] = total;
        const int64_t sz = (int64_t)bs * bs * (hp[b] == BJ_P16 ? 2 : hp[b] == BJ_P32 ? 4 : 8);
        total += (sz + 15) / 16 * 16;
    }
    J->bstore = mk((size_t)total);
    if (!J->bstore) return set_error(MXL_ERR_OUT_OF_MEMORY, "block Jacobi storage");
    J->bstore_bytes = total;
    if ((e = hipMemcpyAsync(J->boff->p, ho.data(), (size_t)nb * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = bj_pack(bs, nb, (const double *)tmp->p, (const int *)J->bprec->p, (const int64_t *)J->boff->p,
                     (unsigned char *)J->bstore->p, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, std::string("block Jacobi packing: ") + hipGetErrorString(e));
    auto *op = new mxl_op;
    op->kind = MXL_OP_JACOBI;
    op->jac = J;
    *Pout = op;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

namespace {

BufPtr dev_buf(size_t bytes) {
    auto d = std::make_shared<DevBuf>();
    if (hipMalloc(&d->p, bytes ? bytes : 16) != hipSuccess) return BufPtr();
    d->bytes = bytes;
    d->owned = true;
    return d;
}

// Supervariable agglomeration: runs of rows with one column set (same[i]:
// row i continues the run of row i - 1), each cut into pieces of at most
// max_bs rows, packed in row order into blocks of at most max_bs rows (a
// piece that does not fit starts the next block).
std::vector<int32_t> agglomerate(const std::vector<unsigned char> &same, int max_bs) {
    const int64_t n = (int64_t)same.size();
    std::vector<int32_t> bp{0};
    int64_t fill = 0;
    for (int64_t i = 0; i < n;) {
        int64_t e = i + 1;
        while (e < n && same[(size_t)e]) ++e;
        for (int64_t p = i; p < e; p += max_bs) {
            const int64_t len = std::min<int64_t>(max_bs, e - p);
            if (fill > 0 && fill + len > max_bs) {
                bp.push_back((int32_t)p);
                fill = 0;
            }
            fill += len;
        }
        i = e;
    }
    bp.push_back((int32_t)n);
    return bp;
}

// Generation over given boundaries (block sizes 1..32): per size class a
// list of its blocks and one launch of the class's elimination kernel, then
// the precision read-back, the 16-byte-aligned offsets and the packing.
mxl_status bj_generate_var(const std::shared_ptr<MatrixImpl> &A, std::vector<int32_t> bp, int adaptive,
                           double accuracy, mxl_op **Pout) {
    hipStream_t s = A->ctx->stream;
    const int64_t nb = (int64_t)bp.size() - 1;
    static const int kClass[6] = {1, 2, 4, 8, 16, 32};
    std::vector<int> list;
    list.reserve((size_t)nb);
    int64_t cstart[7] = {0};
    std::vector<int64_t> toff((size_t)nb + 1, 0);
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t m = bp[(size_t)b + 1] - bp[(size_t)b];
        toff[(size_t)b + 1] = toff[(size_t)b] + m * m;
    }
    for (int c = 0; c < 6; ++c) {
        cstart[c] = (int64_t)list.size();
        const int lo = c == 0 ? 1 : kClass[c - 1] + 1, hi = kClass[c];
        for (int64_t b = 0; b < nb; ++b) {
            const int m = bp[(size_t)b + 1] - bp[(size_t)b];
            if (m >= lo && m <= hi) list.push_back((int)b);
        }
    }
    cstart[6] = (int64_t)list.size();
    auto J = std::make_shared<JacobiImpl>();
    J->A = A;
    J->block = true;
    J->var = true;
    J->bs = 0;
    J->nblocks = nb;
    BufPtr dlist = dev_buf(list.size() * 4), dtoff = dev_buf((size_t)(nb + 1) * 8),
           tmp = dev_buf((size_t)toff[(size_t)nb] * 8), bad = dev_buf(4);
    J->bptr_d = dev_buf((size_t)(nb + 1) * 4);
    J->rblk = dev_buf((size_t)A->nrows * 4);
    J->bcond = dev_buf((size_t)nb * 8);
    J->bprec = dev_buf((size_t)nb * 4);
    J->boff = dev_buf((size_t)nb * 8);
    if (!dlist || !dtoff || !tmp || !bad || !J->bptr_d || !J->rblk || !J->bcond || !J->bprec || !J->boff)
        return set_error(MXL_ERR_OUT_OF_MEMORY, "block Jacobi workspace");
    hipError_t e;
    const int none = INT_MAX;
    if ((e = hipMemcpyAsync(dlist->p, list.data(), list.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(dtoff->p, toff.data(), (size_t)(nb + 1) * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(J->bptr_d->p, bp.data(), (size_t)(nb + 1) * 4, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(bad->p, &none, 4, hipMemcpyHostToDevice, s)) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, std::string("block Jacobi upload: ") + hipGetErrorString(e));
    const int *rp = (const int *)A->row_ptr->p, *col = (const int *)A->col->p;
    const double *val = (const double *)A->val->p;
    double *inv = (double *)tmp->p, *cond = (double *)J->bcond->p;
    int *prec = (int *)J->bprec->p, *badp = (int *)bad->p;
    for (int c = 0; c < 6; ++c) {
        const int64_t cnt = cstart[c + 1] - cstart[c];
        if (cnt == 0) continue;
        const BlockSel sel{(const int *)dlist->p + cstart[c], (const int *)J->bptr_d->p,
                           (const int64_t *)dtoff->p};
        switch (kClass[c]) {
        case 32:
            hipLaunchKernelGGL((k_bj_invert1<32, true>), dim3((unsigned)cnt), dim3(kWave), 0, s, A->nrows, rp, col,
                               val, adaptive, accuracy, inv, cond, prec, badp, sel);
            break;
#define MXL_BJV(BSV)                                                                                         \
    case BSV:                                                                                                \
        hipLaunchKernelGGL((k_bj_invert<BSV, true>), dim3((unsigned)((cnt + kWave / BSV - 1) / (kWave / BSV))), \
                           dim3(kWave), 0, s, A->nrows, rp, col, val, adaptive, accuracy, inv, cond, prec, badp,  \
                           sel, cnt);                                                                        \
        break;
            MXL_BJV(1) MXL_BJV(2) MXL_BJV(4) MXL_BJV(8) MXL_BJV(16)
#undef MXL_BJV
        }
        if ((e = hipGetLastError()) != hipSuccess)
            return set_error(MXL_ERR_DEVICE, std::string("block inversion: ") + hipGetErrorString(e));
    }
    hipLaunchKernelGGL(k_bj_rowmap, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, nb,
                       (const int *)J->bptr_d->p, (int *)J->rblk->p);
    int hb = INT_MAX;
    std::vector<int> hp((size_t)nb);
    if ((e = hipGetLastError()) != hipSuccess ||
        hipMemcpyAsync(&hb, bad->p, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hp.data(), J->bprec->p, (size_t)nb * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "block inversion read-back");
    if (hb != INT_MAX) {
        char msg[96];
        snprintf(msg, sizeof msg, "diagonal block %d is singular", hb);
        return set_error(MXL_ERR_ZERO_DIAG, msg);
    }
    std::vector<int64_t> ho((size_t)nb);
    int64_t total = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int m = bp[(size_t)b + 1] - bp[(size_t)b];
        ho[(size_t)b] = total;
        total += (int64_t)m * bjv_chunks(m, hp[(size_t)b]) * 16;
    }
    J->bstore = dev_buf((size_t)total);
    if (!J->bstore) return set_error(MXL_ERR_OUT_OF_MEMORY, "block Jacobi storage");
    J->bstore_bytes = total;
    if ((e = hipMemcpyAsync(J->boff->p, ho.data(), (size_t)nb * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "block Jacobi offsets");
    hipLaunchKernelGGL(k_bj_pack_var, dim3((unsigned)nb), dim3(kWave), 0, s, nb, (const int *)J->bptr_d->p,
                       (const int64_t *)dtoff->p, (const double *)tmp->p, (const int *)J->bprec->p,
                       (const int64_t *)J->boff->p, (unsigned char *)J->bstore->p);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, std::string("block Jacobi packing: ") + hipGetErrorString(e));
    J->bptr_h = std::move(bp);
    auto *op = new mxl_op;
    op->kind = MXL_OP_JACOBI;
    op->jac = J;
    *Pout = op;
    return MXL_OK;
}

}  // namespace

extern "C" mxl_status mxl_bjacobi_generate_var(const mxl_op *Aop, int64_t nblocks, const int32_t *bptr_host,
                                               int32_t max_block_size, int32_t adaptive, double accuracy,
                                               mxl_op **Pout) try {
    if (!Aop || !Pout || Aop->kind != MXL_OP_MATRIX)
        return set_error(MXL_ERR_INVALID_ARG, "matrix operator and output required");
    *Pout = nullptr;
    const auto &A = Aop->mat;
    if (A->nrows != A->ncols) return set_error(MXL_ERR_NOT_IMPLEMENTED, "block Jacobi needs a square matrix");
    if (A->dtype != MXL_F64) return set_error(MXL_ERR_NOT_IMPLEMENTED, "block Jacobi needs an FP64 matrix");
    if (A->format == MXL_FMT_STENCIL)
        return set_error(MXL_ERR_NOT_IMPLEMENTED, "block Jacobi needs stored matrix rows");
    if (A->nrows == 0) return set_error(MXL_ERR_INVALID_ARG, "empty matrix");
    if (!(accuracy >= 0.0)) return set_error(MXL_ERR_INVALID_ARG, "accuracy must be >= 0");
    if (accuracy == 0.0) accuracy = 0.1;
    const int64_t n = A->nrows;
    DeviceScope ds(A->ctx->device);
    hipStream_t s = A->ctx->stream;
    std::vector<int32_t> bp;
    if (bptr_host) {
        if (nblocks < 1 || nblocks > n) return set_error(MXL_ERR_INVALID_ARG, "1 <= nblocks <= nrows required");
        bp.assign(bptr_host, bptr_host + nblocks + 1);
        if (bp[0] != 0 || bp[(size_t)nblocks] != n)
            return set_error(MXL_ERR_INVALID_ARG, "block boundaries must run from 0 to nrows");
        for (int64_t b = 0; b < nblocks; ++b) {
            const int64_t m = (int64_t)bp[(size_t)b + 1] - bp[(size_t)b];
            if (m < 1 || m > kBjMax) {
                char msg[112];
                snprintf(msg, sizeof msg, "block %lld has %lld rows (1 to %d allowed)", (long long)b,
                         (long long)m, kBjMax);
                return set_error(MXL_ERR_INVALID_ARG, msg);
            }
        }
    } else {
        if (max_block_size < 1 || max_block_size > kBjMax)
            return set_error(MXL_ERR_INVALID_ARG, "max_block_size must be 1..32");
        BufPtr same = dev_buf((size_t)n);
        if (!same) return set_error(MXL_ERR_OUT_OF_MEMORY, "supervariable flags");
        hipLaunchKernelGGL(k_bj_same_prev, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                           (const int *)A->row_ptr->p, (const int *)A->col->p, (unsigned char *)same->p);
        std::vector<unsigned char> h((size_t)n);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h.data(), same->p, (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return set_error(MXL_ERR_DEVICE, "supervariable detection");
        bp = agglomerate(h, max_block_size);
    }
    return bj_generate_var(A, std::move(bp), adaptive ? 1 : 0, accuracy, Pout);
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_bjacobi_blocks(const mxl_op *Pop, int32_t *bptr_host) try {
    if (!Pop || Pop->kind != MXL_OP_JACOBI || !Pop->jac->block || !bptr_host)
        return set_error(MXL_ERR_INVALID_ARG, "block-Jacobi operator and output required");
    const JacobiImpl &J = *Pop->jac;
    if (J.var) {
        std::copy(J.bptr_h.begin(), J.bptr_h.end(), bptr_host);
    } else {
        for (int64_t b = 0; b <= J.nblocks; ++b) bptr_host[b] = (int32_t)std::min<int64_t>(b * J.bs, J.A->nrows);
    }
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_bjacobi_info(const mxl_op *Pop, int64_t *nblocks, double *cond_host,
                                       int32_t *precision_host, double *inv_host, int64_t *storage_bytes) try {
    if (!Pop || Pop->kind != MXL_OP_JACOBI || !Pop->jac->block)
        return set_error(MXL_ERR_INVALID_ARG, "not a block-Jacobi operator");
    const JacobiImpl &J = *Pop->jac;
    DeviceScope ds(J.A->ctx->device);
    hipStream_t s = J.A->ctx->stream;
    const int64_t nb = J.nblocks, bs = J.bs, n = J.A->nrows;
    if (nblocks) *nblocks = nb;
    if (storage_bytes) *storage_bytes = J.bstore_bytes;
    if (cond_host && hipMemcpyAsync(cond_host, J.bcond->p, (size_t)nb * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "copy condition numbers");
    std::vector<int> hp((size_t)nb);
    if (hipMemcpyAsync(hp.data(), J.bprec->p, (size_t)nb * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "copy precisions");
    std::vector<unsigned char> store;
    std::vector<int64_t> ho;
    if (inv_host) {
        store.resize((size_t)J.bstore_bytes);
        ho.resize((size_t)nb);
        if (hipMemcpyAsync(store.data(), J.bstore->p, store.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(ho.data(), J.boff->p, (size_t)nb * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
            return set_error(MXL_ERR_DEVICE, "copy inverses");
    }
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(MXL_ERR_DEVICE, "block Jacobi read-back");
    if (precision_host)
        for (int64_t b = 0; b < nb; ++b) precision_host[b] = hp[b];
    if (inv_host) {  // packed m x m per block, as FP64
        int64_t o = 0;
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t m = J.var ? J.bptr_h[(size_t)b + 1] - J.bptr_h[(size_t)b] : std::min(bs, n - b * bs);
            // elements per stored row: bs (uniform) or whole 16-byte chunks (variable)
            const int64_t ld = J.var ? (int64_t)bjv_chunks((int)m, hp[b]) * (hp[b] == BJ_P16 ? 8 : hp[b] == BJ_P32 ? 4 : 2)
                                     : bs;
            const unsigned char *base = store.data() + ho[b];
            for (int64_t i = 0; i < m; ++i)
                for (int64_t jj = 0; jj < m; ++jj) {
                    const int64_t k = i * ld + jj;
                    double x;
                    if (hp[b] == BJ_P16) {
                        _Float16 h;
                        std::memcpy(&h, base + 2 * k, 2);
                        x = (double)h;
                    } else if (hp[b] == BJ_P32) {
                        float f;
                        std::memcpy(&f, base + 4 * k, 4);
                        x = f;
                    } else {
                        std::memcpy(&x, base + 8 * k, 8);
                    }
                    inv_host[o++] = x;
                }
        }
    }
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}
