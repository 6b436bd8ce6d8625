// spmv.hip -- sparse matrix-vector product y = alpha*A*x + beta*y for CSR
// (scalar, vector-W, merge-path), COO (segmented reduction), ELL (plain and
// LDS-staged x window) and HYB (ELL + COO tail), with an optional fused dot
// product w.y and the setup kernels (partitioning, format conversion,
// validation, Jacobi extraction).
//
// The apply semantics are the simple and advanced applications of a linear
// operator (Sec. 2.2.2 and Sec. 4.2 of the paper); the kernel designs are
// this library's own, written for wave64 CDNA4: every kernel is
// HBM-bandwidth bound (about 0.17 flop per byte in FP64), so the designs aim
// at coalesced, wide, streaming loads of the matrix arrays and keep the
// gathered x in cache.  No MFMA: this is not a dense contraction.
#include <climits>

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace mxl {

template <typename V>
struct SpmvK {
    const V *x;
    V *y;
    V alpha, beta;
    int beta_zero;
    const int *stop;  // nullable: skip all work when *stop != 0
    const V *w;       // nullable: fused dot w.y, one partial per workgroup
    double *partials;
    int slot_base;
};

template <typename V>
__device__ __forceinline__ V combine(const SpmvK<V> &p, V acc, int64_t row) {
    return p.beta_zero ? p.alpha * acc : p.alpha * acc + p.beta * p.y[row];
}

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}

// ------------------------------------------------------------ CSR scalar
// One lane per row.  Good for very short rows; long rows serialise.
template <typename V, bool DOT>
__global__ __launch_bounds__(kWG) void k_csr_scalar(int64_t n, const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    const V *__restrict__ val, SpmvK<V> p) {
    if (p.stop && *p.stop) return;
    const int L = blockIdx.x;
    const int64_t ngroups = (n + kWG - 1) / kWG;
    int64_t g0, g1;
    int gs;
    band_walk(ngroups, blockIdx.x, gridDim.x, g0, g1, gs);
    double dacc = 0.0;
    for (int64_t g = g0; g < g1; g += gs) {
        int64_t row = g * kWG + threadIdx.x;
        if (row >= n) continue;
        int k0 = rp[row], k1 = rp[row + 1];
        V acc = 0;
        for (int k = k0; k < k1; ++k) acc += ld_stream(val + k) * p.x[ld_stream(col + k)];
        V out = combine(p, acc, row);
        p.y[row] = out;
        if (DOT) dacc += (double)p.w[row] * (double)out;
    }
    if (DOT) {
        double v[1] = {dacc};
        publish<1>(v, p.partials, p.slot_base + L);
    }
}

// ------------------------------------------------------------ CSR vector
// W lanes per row (W = 2..64), lanes stride through the row so a group's
// loads are contiguous; the W partial sums are combined by a shuffle tree.
// Each lane group keeps kVecU rows in flight: the row bounds, then the
// first W entries of all kVecU rows are loaded before any x is gathered, so
// a wave has several independent memory requests outstanding instead of one
// dependent chain per row.
constexpr int kVecU = 4;

template <typename V, int W, bool DOT>
__global__ __launch_bounds__(kWG) void k_csr_vector(int64_t n, const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    const V *__restrict__ val, SpmvK<V> p) {
    if (p.stop && *p.stop) return;
    constexpr int RPG = kWG / W;  // rows per workgroup step
    const int L = blockIdx.x;
    const int64_t ngroups = (n + RPG - 1) / RPG;
    int64_t g0, g1;
    int gs;
    band_walk(ngroups, blockIdx.x, gridDim.x, g0, g1, gs);
    const int lane = threadIdx.x % W, sub = threadIdx.x / W;
    double dacc = 0.0;
    for (int64_t g = g0; g < g1; g += (int64_t)gs * kVecU) {
        int k0[kVecU], k1[kVecU];
#pragma unroll
        for (int u = 0; u < kVecU; ++u) {
            const int64_t gu = g + (int64_t)u * gs;
            const int64_t row = gu * RPG + sub;
            const bool ok = gu < g1 && row < n;
            k0[u] = ok ? rp[row] : 0;
            k1[u] = ok ? rp[row + 1] : 0;
        }
        // first EPL entries of every row in flight, then the rest of long rows
        constexpr int EPL = 1;
        int c[kVecU][EPL];
        V v[kVecU][EPL];
#pragma unroll
        for (int u = 0; u < kVecU; ++u)
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int k = k0[u] + lane + e * W;
                const bool in = k < k1[u];
                c[u][e] = in ? ld_stream(col + k) : -1;
                v[u][e] = in ? ld_stream(val + k) : (V)0;
            }
        V acc[kVecU];
#pragma unroll
        for (int u = 0; u < kVecU; ++u) {
            acc[u] = 0;
#pragma unroll
            for (int e = 0; e < EPL; ++e)
                if (c[u][e] >= 0) acc[u] += v[u][e] * p.x[c[u][e]];
        }
#pragma unroll
        for (int u = 0; u < kVecU; ++u)  // rows longer than EPL*W
            for (int k = k0[u] + lane + EPL * W; k < k1[u]; k += W) acc[u] += ld_stream(val + k) * p.x[ld_stream(col + k)];
#pragma unroll
        for (int u = 0; u < kVecU; ++u) {
#pragma unroll
            for (int off = W / 2; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off, W);
            const int64_t gu = g + (int64_t)u * gs;
            const int64_t row = gu * RPG + sub;
            if (gu < g1 && row < n && lane == 0) {
                V out = combine(p, acc[u], row);
                p.y[row] = out;
                if (DOT) dacc += (double)p.w[row] * (double)out;
            }
        }
    }
    if (DOT) {
        double vv[1] = {dacc};
        publish<1>(vv, p.partials, p.slot_base + L);
    }
}

// ------------------------------------------------------- row-block CSR
// Rows are cut (once, at conversion) into blocks of at most kStreamRows
// consecutive rows holding at most kStreamK*64 nonzeros; a row longer than
// that forms a block of its own.  Block b is described by (first row, first
// nonzero) in blk[b] (blk[nblk] = (n, nnz)).  One wave takes a block: its
// lanes load the block's nonzeros as kStreamK fully coalesced, independent
// loads, gather x, and park the products in the wave's LDS slice; then lane
// l sums the products of row first+l in order.  A long row is swept by the
// whole wave and reduced by shuffles.  No workgroup barrier is involved:
// every wave walks its own blocks.
constexpr int kStreamK = 8;
constexpr int kStreamRows = 63;  // a lane reads the next row's start from its neighbour

template <typename V, bool DOT>
__global__ __launch_bounds__(kWG) void k_csr_stream(int64_t nblk, const int2 *__restrict__ blk,
                                                    const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    const V *__restrict__ val, SpmvK<V> p) {
    if (p.stop && *p.stop) return;
    __shared__ V s_prod[kWG / kWave][kStreamK * kWave];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    constexpr int WPG = kWG / kWave;
    // walkers: 4 waves per workgroup; when the grid is a multiple of 8 the
    // walker id keeps the workgroup's XCD (blockIdx % 8) in its low bits
    const int G = (int)gridDim.x, nw = G * WPG;
    const int vid = (G % kNumXcd == 0)
                        ? ((int)(blockIdx.x / kNumXcd) * WPG + wid) * kNumXcd + (int)(blockIdx.x % kNumXcd)
                        : (int)blockIdx.x * WPG + wid;
    int64_t b0, b1;
    int bs;
    band_walk(nblk, vid, nw, b0, b1, bs);
    V *sp = s_prod[wid];
    double dacc = 0.0;
    int2 d0 = make_int2(0, 0), d1 = make_int2(0, 0);
    if (b0 < b1) {
        d0 = blk[b0];
        d1 = blk[b0 + 1];
    }
    for (int64_t b = b0; b < b1; b += bs) {
        // descriptor of the next block, loaded while this one is processed
        const int64_t bn = b + bs;
        int2 e0 = make_int2(0, 0), e1 = make_int2(0, 0);
        if (bn < b1) {
            e0 = blk[bn];
            e1 = blk[bn + 1];
        }
        const int r0 = d0.x, k0 = d0.y, nr = d1.x - d0.x, k1 = d1.y;
        if (k1 - k0 > kStreamK * kWave) {  // one long row, kStreamK loads per lane in flight
            V acc = 0;
            for (int kb = k0; kb < k1; kb += kStreamK * kWave) {
                int c[kStreamK];
                V v[kStreamK];
#pragma unroll
                for (int j = 0; j < kStreamK; ++j) {
                    const int k = kb + lane + kWave * j;
                    const bool in = k < k1;
                    c[j] = in ? ld_stream(col + k) : -1;
                    v[j] = in ? ld_stream(val + k) : (V)0;
                }
                // same order as one entry at a time: k = lane, lane + 64, ...
#pragma unroll
                for (int j = 0; j < kStreamK; ++j)
                    if (c[j] >= 0) acc += v[j] * p.x[c[j]];
            }
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
            if (lane == 0) {
                const V out = combine(p, acc, r0);
                p.y[r0] = out;
                if (DOT) dacc += (double)p.w[r0] * (double)out;
            }
        } else {
            const int rs = lane <= nr ? rp[r0 + lane] : 0;
            int c[kStreamK];
            V v[kStreamK];
#pragma unroll
            for (int j = 0; j < kStreamK; ++j) {
                const int k = k0 + lane + kWave * j;
                const bool in = k < k1;
                c[j] = in ? ld_stream(col + k) : -1;
                v[j] = in ? ld_stream(val + k) : (V)0;
            }
#pragma unroll
            for (int j = 0; j < kStreamK; ++j) sp[lane + kWave * j] = c[j] >= 0 ? v[j] * p.x[c[j]] : (V)0;
            // each row of the block gets g = 2^lg lanes (as many as 64 / nr
            // allows, at most 8): lane l sums every g-th product of row l >> lg
            // from offset l & (g - 1), and the g partial sums meet by shuffles
            const int lg = nr <= 8 ? 3 : (nr <= 16 ? 2 : (nr <= 32 ? 1 : 0));
            const int myrow = lane >> lg, part = lane & ((1 << lg) - 1);
            const int rs_m = __shfl(rs, myrow < kWave ? myrow : kWave - 1, kWave);
            const int re_m = __shfl(rs, myrow + 1 < kWave ? myrow + 1 : kWave - 1, kWave);
            // products visible to the other lanes of this wave (LDS is in order per wave)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            V acc = 0;
            if (myrow < nr)
                for (int k = rs_m - k0 + part; k < re_m - k0; k += 1 << lg) acc += sp[k];
            for (int off = 1; off < (1 << lg); off <<= 1) acc += __shfl_xor(acc, off, kWave);
            if (myrow < nr && part == 0) {
                const int64_t row = (int64_t)r0 + myrow;
                const V out = combine(p, acc, row);
                p.y[row] = out;
                if (DOT) dacc += (double)p.w[row] * (double)out;
            }
            __builtin_amdgcn_wave_barrier();  // reads done before the next block's writes
        }
        d0 = e0;
        d1 = e1;
    }
    if (DOT) {
        double vv[1] = {dacc};
        publish<1>(vv, p.partials, p.slot_base + (int)blockIdx.x);
    }
}

// ------------------------------------------------------- merge path CSR
// The (row ends) x (nonzeros) merge sequence of n + nnz items is cut into
// tiles of ITEMS = 256*IPT items; coordinates of every tile boundary are
// precomputed (k_merge_partition).  A tile stages its products and row ends
// in LDS with coalesced loads, each thread walks IPT consecutive items, and
// rows crossing thread or tile boundaries are completed by deterministic
// carry chains (in LDS within a tile, k_carry_fixup across tiles).
struct Carry {
    int32_t row;  // -1: none
    int32_t pad;
    double val;
};

constexpr int kMergeIPT = 6;
constexpr int kMergeItems = kWG * kMergeIPT;

__global__ void k_merge_partition(int64_t n, int64_t nnz, const int *__restrict__ rp, int64_t ntiles,
                                  int2 *__restrict__ part) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > ntiles) return;
    int64_t d = b * kMergeItems;
    if (d > n + nnz) d = n + nnz;
    // i = number of rows m whose end item (position m + rp[m+1]) precedes d
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (mid + rp[mid + 1] < d) lo = mid + 1;
        else hi = mid;
    }
    part[b] = make_int2((int)lo, (int)(d - lo));
}

template <typename V, bool DOT>
__global__ __launch_bounds__(kWG) void k_csr_merge(int64_t n, const int *__restrict__ rp,
                                                   const int *__restrict__ col,
                                                   const V *__restrict__ val,
                                                   const int2 *__restrict__ part, int64_t ntiles,
                                                   Carry *__restrict__ carries, SpmvK<V> p) {
    if (p.stop && *p.stop) return;
    __shared__ int s_end[kMergeItems + 1];
    __shared__ V s_prod[kMergeItems];
    __shared__ V s_out[kMergeItems];
    __shared__ int s_crow[kWG];
    __shared__ V s_cval[kWG];
    const int tid = threadIdx.x;
    const int L = blockIdx.x;
    int64_t t0, t1;
    int ts;
    band_walk(ntiles, blockIdx.x, gridDim.x, t0, t1, ts);
    double dacc = 0.0;
    for (int64_t tile = t0; tile < t1; tile += ts) {
        const int2 c0 = part[tile], c1 = part[tile + 1];
        const int r0 = c0.x, k0 = c0.y, r1 = c1.x, k1 = c1.y;
        const int nr = r1 - r0, nk = k1 - k0;
        for (int i = tid; i <= nr; i += kWG) s_end[i] = (r0 + i < n) ? rp[r0 + i + 1] : INT_MAX;
#pragma unroll
        for (int u = 0; u < kMergeIPT; ++u) {
            int j = u * kWG + tid;
            if (j < nk) {
                int k = k0 + j;
                s_prod[j] = ld_stream(val + k) * p.x[ld_stream(col + k)];
            }
        }
        __syncthreads();
        const int total = nr + nk;
        int d = tid * kMergeIPT;
        if (d > total) d = total;
        int dend = d + kMergeIPT;
        if (dend > total) dend = total;
        int lo = d - nk > 0 ? d - nk : 0, hi = d < nr ? d : nr;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (mid + (s_end[mid] - k0) < d) lo = mid + 1;
            else hi = mid;
        }
        int i = lo, j = d - lo;
        V acc = 0;
        int first_row = -1;
        V first_val = 0;
        for (int step = d; step < dend; ++step) {
            if (i < nr && s_end[i] - k0 <= j) {
                if (first_row < 0) { first_row = i; first_val = acc; }
                else s_out[i] = acc;
                acc = 0;
                ++i;
            } else {
                acc += s_prod[j];
                ++j;
            }
        }
        s_crow[tid] = i;
        s_cval[tid] = acc;
        __syncthreads();
        if (first_row >= 0) {
            V c = 0;
            for (int t2 = tid - 1; t2 >= 0 && s_crow[t2] == first_row; --t2) c += s_cval[t2];
            s_out[first_row] = first_val + c;
        }
        if (tid == 0) {
            V c = 0;
            for (int t2 = kWG - 1; t2 >= 0 && s_crow[t2] == nr; --t2) c += s_cval[t2];
            Carry cr;
            cr.row = (r1 < n) ? r1 : -1;
            cr.pad = 0;
            cr.val = (double)c;
            carries[tile] = cr;
            if (DOT && r1 < n) dacc += (double)p.w[r1] * (double)(p.alpha * c);
        }
        __syncthreads();
        for (int ii = tid; ii < nr; ii += kWG) {
            int64_t row = r0 + ii;
            V out = combine(p, s_out[ii], row);
            p.y[row] = out;
            if (DOT) dacc += (double)p.w[row] * (double)out;
        }
        __syncthreads();
    }
    if (DOT) {
        double v[1] = {dacc};
        publish<1>(v, p.partials, p.slot_base + L);
    }
}

// ------------------------------------------------------------------ COO
// Wave-level COO: tiles of kCooWaveItems consecutive triplets, one wave per
// tile, no workgroup barrier.  The wave loads its tile with coalesced loads
// (lane l takes items l, l+64, ...: each gather then covers 64
// consecutive items, a few rows' neighbourhoods), parks rows and products
// in its LDS slice, and lane l then walks items 8l..8l+7 in order (taking
// items 8l.. straight from memory instead spreads every gather over the
// whole tile: 322 us against 218 us): rows that end inside
// the lane are written at once; the partial sum of the lane's last row is
// combined across lanes by a segmented inclusive scan (keys = rows, which
// are sorted, so equal keys are contiguous).  The row still open at the end
// of the tile is handed to k_carry_fixup.  Rows without entries are written
// by the lane that sees the row index jump over them (not in ACC mode,
// which accumulates into y: the HYB tail).
constexpr int kCooWaveIPL = 8;                        // items per lane
constexpr int kCooWaveItems = kWave * kCooWaveIPL;    // items per wave tile

template <typename V, bool DOT, bool ACC>
__global__ __launch_bounds__(kWG) void k_coo_wave(int64_t n, int64_t nnz, const int *__restrict__ row,
                                                  const int *__restrict__ col,
                                                  const V *__restrict__ val, int64_t ntiles,
                                                  Carry *__restrict__ carries, SpmvK<V> p) {
    if (p.stop && *p.stop) return;
    constexpr int WPG = kWG / kWave;
    __shared__ int s_row[WPG][kCooWaveItems + 4];  // + the row after the tile; rows 16-byte aligned
    __shared__ V s_prod[WPG][kCooWaveItems];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int G = (int)gridDim.x, nw = G * WPG;
    const int vid = (G % kNumXcd == 0)
                        ? ((int)(blockIdx.x / kNumXcd) * WPG + wid) * kNumXcd + (int)(blockIdx.x % kNumXcd)
                        : (int)blockIdx.x * WPG + wid;
    int64_t t0, t1;
    int ts;
    band_walk(ntiles, vid, nw, t0, t1, ts);
    int *sr = s_row[wid];
    V *sv = s_prod[wid];
    double dacc = 0.0;
    const int nrow = (int)n;
    auto emit = [&](int r, V acc) {  // y[r] from a complete in-tile sum
        const V out = ACC ? p.y[r] + p.alpha * acc : combine(p, acc, r);
        p.y[r] = out;
        if (DOT) dacc += (double)p.w[r] * (double)(ACC ? p.alpha * acc : out);
    };
    for (int64_t tile = t0; tile < t1; tile += ts) {
        const int64_t e0 = tile * kCooWaveItems;
        const int ne = (int)((nnz - e0) < kCooWaveItems ? (nnz - e0) : kCooWaveItems);
        int rr[kCooWaveIPL], cc[kCooWaveIPL];
        V vv[kCooWaveIPL];
#pragma unroll
        for (int j = 0; j < kCooWaveIPL; ++j) {
            const int i = lane + kWave * j;
            const bool in = i < ne;
            rr[j] = in ? ld_stream(row + e0 + i) : 0;
            cc[j] = in ? ld_stream(col + e0 + i) : -1;
            vv[j] = in ? ld_stream(val + e0 + i) : (V)0;
        }
        const int next = (e0 + ne < nnz) ? row[e0 + ne] : nrow;  // row after the tile ("all end" at nnz)
#pragma unroll
        for (int j = 0; j < kCooWaveIPL; ++j) {
            const int i = lane + kWave * j;
            if (i < ne) {
                sr[i] = rr[j];
                sv[i] = vv[j] * p.x[cc[j]];
            }
        }
        if (lane == 0) sr[ne] = next;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int j0 = lane * kCooWaveIPL;
        const int j1 = j0 + kCooWaveIPL < ne ? j0 + kCooWaveIPL : ne;
        if (!ACC && e0 == 0 && lane == 0 && ne > 0)  // rows before the first entry
            for (int g = 0; g < sr[0]; ++g) p.y[g] = combine(p, (V)0, g);
        // walk: rows that start and end inside the lane are final; the first
        // row of the lane (which may have started earlier) is held back
        // the lane's eight items come out of LDS as 16-byte vectors, all
        // issued before the walk (items past the tile's end are read but
        // never used): 280 -> 218 us on the 128^3 27-point matrix against
        // one dependent LDS read per item, 260 us four items at a time
        const int cnt = j1 - j0;
        constexpr int PV = 16 / (int)sizeof(V);
        typedef V VP __attribute__((ext_vector_type(PV)));
        typedef int I4 __attribute__((ext_vector_type(4)));
        int rw[kCooWaveIPL];
        V pw[kCooWaveIPL];
        int rlast = 0;
        if (cnt > 0) {
#pragma unroll
            for (int h = 0; h < kCooWaveIPL; h += 4) {
                const I4 t = *(const I4 *)(sr + j0 + h);
#pragma unroll
                for (int e = 0; e < 4; ++e) rw[h + e] = t[e];
            }
#pragma unroll
            for (int h = 0; h < kCooWaveIPL; h += PV) {
                const VP t = *(const VP *)(sv + j0 + h);
#pragma unroll
                for (int e = 0; e < PV; ++e) pw[h + e] = t[e];
            }
            rlast = sr[j1];  // row of the item after the lane's last
        }
        V acc = 0;
        int head_row = -1;
        V head_val = 0;
        bool at_start = true;
        int rend = 0;  // row of the lane's last item
#pragma unroll
        for (int j = 0; j < kCooWaveIPL; ++j) {
            if (j >= cnt) break;
            const int r = rw[j];
            rend = r;
            acc += pw[j];
            const int rn = j + 1 < cnt ? rw[j + 1] : rlast;
            if (rn != r) {
                if (!ACC) {
                    const int last = rn < nrow ? rn : nrow;
                    for (int g = r + 1; g < last; ++g) p.y[g] = combine(p, (V)0, g);
                }
                if (at_start) {
                    head_row = r;
                    head_val = acc;
                } else {
                    emit(r, acc);
                }
                acc = 0;
                at_start = false;
            }
        }
        // lane tails: the open row at the lane's end and its partial sum
        const bool open = cnt > 0 && rlast == rend;
        int key = open ? rend : -1 - lane;  // closed lanes never chain
        V tail = open ? acc : (V)0;
        // segmented inclusive scan of the tails over lanes
        V scan = tail;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const V up = __shfl_up(scan, d, kWave);
            const int ku = __shfl_up(key, d, kWave);
            if (lane >= d && ku == key) scan += up;
        }
        // carry into this lane's head row: the previous lane's scan if its
        // open row is the head row
        const V prev_scan = __shfl_up(scan, 1, kWave);
        const int prev_key = __shfl_up(key, 1, kWave);
        if (head_row >= 0) {
            const V cin = (lane > 0 && prev_key == head_row) ? prev_scan : (V)0;
            emit(head_row, head_val + cin);
        }
        // the row still open at the tile's end continues in the next tile
        const int last_lane = ne > 0 ? (ne - 1) / kCooWaveIPL : 0;
        const V tile_tail = __shfl(scan, last_lane, kWave);
        const int tile_key = __shfl(key, last_lane, kWave);
        if (lane == 0) {
            Carry cr;
            cr.row = -1;
            cr.pad = 0;
            cr.val = 0.0;
            if (ne > 0 && next == sr[ne - 1]) {
                cr.row = tile_key;
                cr.val = (double)tile_tail;
                if (DOT) dacc += (double)p.w[tile_key] * (double)(p.alpha * tile_tail);
            }
            carries[tile] = cr;
        }
        __builtin_amdgcn_wave_barrier();  // LDS reads done before the next tile's writes
    }
    if (DOT) {
        double vv2[1] = {dacc};
        publish<1>(vv2, p.partials, p.slot_base + (int)blockIdx.x);
    }
}

// Adds the carried partial sums of rows that crossed tile boundaries: one
// thread per tile; the first tile of each run of equal carry rows sums the
// run in tile order (deterministic) and updates y once.
template <typename V>
__global__ __launch_bounds__(kWG) void k_carry_fixup(const Carry *__restrict__ carries,
                                                     int64_t ntiles, SpmvK<V> p) {
    if (p.stop && *p.stop) return;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ntiles) return;
    const int r = carries[g].row;
    if (r < 0) return;
    if (g > 0 && carries[g - 1].row == r) return;
    double s = 0.0;
    for (int64_t g2 = g; g2 < ntiles && carries[g2].row == r; ++g2) s += carries[g2].val;
    p.y[r] = p.y[r] + p.alpha * (V)s;
}

// ------------------------------------------------------------------ ELL
// Slot-major [w][n_pad]: lane i reads slot s of row i at s*n_pad + i, so a
// wave's loads are contiguous.  Padding column -1 is predicated off.  The
// LDS variant first copies the tile's x window [lo, hi] (precomputed per
// 256-row tile) into LDS when it fits, then gathers from LDS.
constexpr int kEllLdsCap = 4096;  // x entries staged per tile (32 KB in FP64)

// Vector types for R consecutive rows of one ELL slot (R = 1, 2, 4); I is
// int (column indices) or short (16-bit offsets col - row).
template <typename I, int R> struct IdxVec { typedef I T __attribute__((ext_vector_type(R))); };
template <typename I> struct IdxVec<I, 1> { typedef I T; };
constexpr short kEll16Pad = -32768;  // padding slot of the 16-bit-offset layout
template <typename V, int R> struct ValVec { typedef V T __attribute__((ext_vector_type(R))); };
template <typename V> struct ValVec<V, 1> { typedef V T; };

template <int R, typename T>
__device__ __forceinline__ auto lane_of(const T &v, int r) {
    if constexpr (R == 1) return v;
    else return v[r];
}

// Each thread owns R consecutive rows (R*256 rows per tile), so one slot's
// column indices and values arrive as one 4R- and one 8R-byte load (16-byte
// loads at R = 4 for indices, 2 x 16 bytes for FP64 values).  U slots of
// loads are issued before their x gathers.
// D16: the slots hold 16-bit offsets d = col - row (kEll16Pad = padding),
// which cuts the index stream from 4 to 2 bytes per slot.
template <typename V, bool DOT, bool LDS, int R, bool D16 = false, bool NB = false>
__global__ __launch_bounds__(kWG) void k_ell(int64_t n, int64_t n_pad, int w,
                                             const void *__restrict__ ecol_,
                                             const V *__restrict__ evals,
                                             const int2 *__restrict__ win, SpmvK<V> p) {
    static_assert(!(LDS && NB), "neighbour reuse is for the global-gather variants");
    if (p.stop && *p.stop) return;
    // slots of loads in flight per batch; with neighbour reuse most slots
    // gather nothing, and 3 FP64 slots of 2 rows keep the kernel at 76
    // registers instead of 84 (128^3 27-point CG product 116 -> 108 us
    // together with the streaming store below)
    constexpr int U = (NB && sizeof(V) == 8 && R == 2) ? 3 : (sizeof(V) == 4 ? 16 : 8) / R;
    typedef typename std::conditional<D16, short, int>::type IT;
    typedef typename IdxVec<IT, R>::T IV;
    const IT *__restrict__ ecol = (const IT *)ecol_;
    typedef typename ValVec<V, R>::T VV;
    __shared__ V s_x[LDS ? kEllLdsCap : 1];
    const int L = blockIdx.x;
    const int64_t ntiles = (n + kWG * R - 1) / (kWG * R);
    int64_t t0, t1;
    int ts;
    band_walk(ntiles, blockIdx.x, gridDim.x, t0, t1, ts);
    double dacc = 0.0;
    const bool yvec = ((uintptr_t)p.y & (sizeof(V) * R - 1)) == 0;  // y aligned for R-row vectors
    for (int64_t tile = t0; tile < t1; tile += ts) {
        const int64_t row0 = tile * kWG * R + (int64_t)threadIdx.x * R;
        bool staged = false;
        int lo = 0;
        if (LDS) {
            int2 wv = win[tile];
            lo = wv.x;
            int span = wv.y - wv.x + 1;
            staged = span > 0 && span <= kEllLdsCap;
            if (staged) {
                for (int j = threadIdx.x; j < span; j += kWG) s_x[j] = p.x[lo + j];
            }
            __syncthreads();
        }
        // rows row0..row0+R-1 < n_pad (n_pad is a multiple of 64).  With NB
        // every lane of the wave runs the slot loop (the shuffles need all
        // lanes); lanes past n load nothing and see padding only.
        const bool live = row0 < n;
        if (NB || live) {
            const IV *cp = (const IV *)(ecol + (live ? row0 : 0));
            const VV *vp = (const VV *)(evals + (live ? row0 : 0));
            // the fused dot's w rows are loaded with the first slots, not
            // after the sums (the dependent load at the tile's end cost
            // 5 us per 128^3 product in the CG loop); w never aliases y
            VV wpre;
            const bool wvec = DOT && R > 1 && live && row0 + R <= n &&
                              ((uintptr_t)p.w & (sizeof(V) * R - 1)) == 0;
            if (wvec) wpre = *(const VV *)(p.w + row0);
            const int64_t stride = n_pad / R;  // one slot, in vector units
            V acc[R];
            int pc[R];  // NB: columns and x values of the previous slot
            V px[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                acc[r] = 0;
                pc[r] = -1;
                px[r] = 0;
            }
            for (int s0 = 0; s0 < w; s0 += U) {
                IV c[U];
                VV v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if ((!NB || live) && s0 + u < w) {
                        c[u] = __builtin_nontemporal_load(cp + (int64_t)(s0 + u) * stride);
                        v[u] = __builtin_nontemporal_load(vp + (int64_t)(s0 + u) * stride);
                    } else {
                        c[u] = (IV)(D16 ? kEll16Pad : -1);
                        v[u] = (VV)(V)0;
                    }
                }
                int ci[U][R];  // column index, -1 for padding
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int e = (int)lane_of<R>(c[u], r);
                        if constexpr (D16) ci[u][r] = e == kEll16Pad ? -1 : (int)(row0 + r) + e;
                        else ci[u][r] = e;
                    }
                V xv[U][R];
                if constexpr (NB) {
                    // Entry (i, s) whose column equals that of entry (i+1, s-1)
                    // takes x from it instead of gathering: row i+1 is the
                    // thread's next row or, for its last row, the first row of
                    // the next lane.  The value moved is x at the compared
                    // column, so the product is unchanged.  Hits are decided
                    // from the columns before any gather is issued.
                    bool hit[U][R];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
#pragma unroll
                        for (int r = 0; r + 1 < R; ++r) {
                            const int q = u == 0 ? pc[r + 1] : ci[u - 1][r + 1];
                            hit[u][r] = ci[u][r] >= 0 && ci[u][r] == q;
                        }
                        const int nq = __shfl_down(u == 0 ? pc[0] : ci[u - 1][0], 1, kWave);
                        hit[u][R - 1] = ci[u][R - 1] >= 0 && ci[u][R - 1] == nq;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            xv[u][r] = ci[u][r] >= 0 && !hit[u][r] ? p.x[ci[u][r]] : (V)0;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
#pragma unroll
                        for (int r = 0; r + 1 < R; ++r)
                            if (hit[u][r]) xv[u][r] = u == 0 ? px[r + 1] : xv[u - 1][r + 1];
                        const V nx = __shfl_down(u == 0 ? px[0] : xv[u - 1][0], 1, kWave);
                        if (hit[u][R - 1]) xv[u][R - 1] = nx;
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        pc[r] = ci[U - 1][r];
                        px[r] = xv[U - 1][r];
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int cc = ci[u][r];
                            xv[u][r] = cc >= 0 ? ((LDS && staged) ? s_x[cc - lo] : p.x[cc]) : (V)0;
                        }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (ci[u][r] >= 0) acc[r] += lane_of<R>(v[u], r) * xv[u][r];
            }
            if (!live) {
                // NB lane past the last row: nothing to store
            } else if (R > 1 && yvec && row0 + R <= n) {
                // the thread's R outputs as one vector store (two half-line
                // stores per line cost twice the write traffic)
                VV yo, yi;
                if (!p.beta_zero) yi = *(const VV *)(p.y + row0);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    V out;
                    if constexpr (R == 1) out = p.beta_zero ? p.alpha * acc[r] : p.alpha * acc[r] + p.beta * yi;
                    else out = p.beta_zero ? p.alpha * acc[r] : p.alpha * acc[r] + p.beta * yi[r];
                    if constexpr (R == 1) yo = out;
                    else yo[r] = out;
                    if (DOT) dacc += (double)(wvec ? lane_of<R>(wpre, r) : p.w[row0 + r]) * (double)out;
                }
                // FP64 outputs stream past the caches (6 us less per 128^3
                // product in the CG loop); FP32 inner solves ran 3 % slower so
                if constexpr (sizeof(V) == 8) __builtin_nontemporal_store(yo, (VV *)(p.y + row0));
                else *(VV *)(p.y + row0) = yo;
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t row = row0 + r;
                    if (row < n) {
                        V out = combine(p, acc[r], row);
                        p.y[row] = out;
                        if (DOT) dacc += (double)p.w[row] * (double)out;
                    }
                }
            }
        }
        if (LDS) __syncthreads();
    }
    if (DOT) {
        double vv[1] = {dacc};
        publish<1>(vv, p.partials, p.slot_base + L);
    }
}

// y = beta*y (alpha*A*x with no stored entries)
template <typename V>
__global__ void k_scale_only(int64_t n, SpmvK<V> p) {
    if (p.stop && *p.stop) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p.y[i] = combine(p, (V)0, i);
}

// ------------------------------------------------------- matrix-free stencil
// Constant-coefficient stencil on an nx x ny x nz grid (x fastest): no
// matrix is stored, so a product moves only x (once, through the caches)
// and y.  The points live on the 3x3x3 cube; point q = 9 (dk+1) + 3 (dj+1) +
// (di+1) is present when bit q of `mask` is set.  Each thread computes one
// point with the cube unrolled at compile time (STAR keeps only the 7
// points with at most one nonzero offset); out-of-grid and absent points
// load the point itself and are discarded by a select, so they never
// multiply x, and no branch separates the loads.
struct StencilK {
    int nx, ny, nz;
    double inv_nx, inv_nxy;  // reciprocals for the index split
    uint32_t mask;
    double c[27];
};

// q = floor(a / b) for 0 <= a < 2^31 from a rounded reciprocal, corrected
// by one step either way.
__device__ __forceinline__ int div_fix(int a, int b, double inv) {
    int q = (int)((double)a * inv);
    if (q * b > a) --q;
    else if ((q + 1) * b <= a) ++q;
    return q;
}

// R consecutive points of one x-line per thread (nx a multiple of R): the
// points share the x values of each (dj, dk) line, so a line costs R + 2
// loads instead of 3 R.  Each point adds its terms in the order of q.
template <typename V, bool DOT, bool STAR, int R>
__global__ __launch_bounds__(kWG) void k_stencil(StencilK sk, SpmvK<V> p) {
    if (p.stop && *p.stop) return;
    // the coefficients go through LDS (broadcast reads) rather than 54
    // scalar registers
    __shared__ V s_c[27];
    if (threadIdx.x < 27) s_c[threadIdx.x] = (V)sk.c[threadIdx.x];
    __syncthreads();
    typedef typename ValVec<V, R>::T VV;
    const int nxy = sk.nx * sk.ny, n = nxy * sk.nz;
    const int64_t ntiles = ((int64_t)n + kWG * R - 1) / (kWG * R);
    int64_t t0, t1;
    int ts;
    band_walk(ntiles, blockIdx.x, gridDim.x, t0, t1, ts);
    double dacc = 0.0;
    const bool yvec = R > 1 && ((uintptr_t)p.y & (sizeof(V) * R - 1)) == 0;
    for (int64_t tile = t0; tile < t1; tile += ts) {
        const int r0 = (int)(tile * kWG * R) + (int)threadIdx.x * R;
        if (r0 >= n) continue;
        const int k = div_fix(r0, nxy, sk.inv_nxy), rem = r0 - k * nxy;
        const int j = div_fix(rem, sk.nx, sk.inv_nx), i0 = rem - j * sk.nx;
        V acc[R];
#pragma unroll
        for (int e = 0; e < R; ++e) acc[e] = 0;
#pragma unroll
        for (int dk = -1; dk <= 1; ++dk)
#pragma unroll
            for (int dj = -1; dj <= 1; ++dj) {
                if (STAR && dj != 0 && dk != 0) continue;
                const bool full = !STAR || (dj == 0 && dk == 0);  // the line holds di = -1, 0, 1
                const bool lin = (dj < 0 ? j > 0 : dj > 0 ? j < sk.ny - 1 : true) &&
                                 (dk < 0 ? k > 0 : dk > 0 ? k < sk.nz - 1 : true);
                const int base = r0 + dj * sk.nx + dk * nxy;
                // x at base-1 .. base+R of this line; a point outside the grid
                // loads x[r0] and is masked below
                V xl[R + 2];
#pragma unroll
                for (int e = -1; e <= R; ++e) {
                    if (!full && (e < 0 || e >= R)) {
                        xl[e + 1] = (V)0;
                        continue;
                    }
                    const bool ok = lin && (e >= 0 || i0 > 0) && (e < R || i0 + R < sk.nx);
                    xl[e + 1] = p.x[ok ? base + e : r0];
                }
#pragma unroll
                for (int di = -1; di <= 1; ++di) {
                    if (!full && di != 0) continue;
                    const int q = 9 * (dk + 1) + 3 * (dj + 1) + (di + 1);
                    const bool present = lin && ((sk.mask >> q) & 1u);
                    const V cq = s_c[q];
#pragma unroll
                    for (int e = 0; e < R; ++e) {
                        const bool ok = present && (di >= 0 || i0 + e > 0) && (di <= 0 || i0 + e < sk.nx - 1);
                        acc[e] += ok ? cq * xl[e + 1 + di] : (V)0;
                    }
                }
            }
        V out[R];
#pragma unroll
        for (int e = 0; e < R; ++e) out[e] = combine(p, acc[e], r0 + e);
        if (yvec) {
            VV yo;
#pragma unroll
            for (int e = 0; e < R; ++e) {
                if constexpr (R == 1) yo = out[e];
                else yo[e] = out[e];
            }
            *(VV *)(p.y + r0) = yo;
        } else {
#pragma unroll
            for (int e = 0; e < R; ++e) p.y[r0 + e] = out[e];
        }
        if (DOT) {
#pragma unroll
            for (int e = 0; e < R; ++e) dacc += (double)p.w[r0 + e] * (double)out[e];
        }
    }
    if (DOT) {
        double vv[1] = {dacc};
        publish<1>(vv, p.partials, p.slot_base + (int)blockIdx.x);
    }
}

// ----------------------------------------------------------- setup kernels
__global__ void k_csr_to_coo(int64_t n, const int *__restrict__ rp, int *__restrict__ row) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = rp[i]; k < rp[i + 1]; ++k) row[k] = (int)i;
}

// 16-bit-offset ELL: slot s of row i holds col - row; *overflow is set
// when some offset does not fit (the layout then cannot hold the matrix).
template <typename V>
__global__ void k_csr_to_ell16(int64_t n, int64_t n_pad, int w, const int *__restrict__ rp,
                               const int *__restrict__ col, const V *__restrict__ val,
                               short *__restrict__ ecol, V *__restrict__ evals, int *overflow) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    int k0 = 0, len = 0;
    if (i < n) { k0 = rp[i]; len = rp[i + 1] - k0; }
    bool bad = false;
    for (int s = 0; s < w; ++s) {
        int64_t o = (int64_t)s * n_pad + i;
        if (s < len) {
            const int64_t d = (int64_t)col[k0 + s] - i;
            bad |= d < -32767 || d > 32767;
            ecol[o] = (short)d;
            evals[o] = val[k0 + s];
        } else {
            ecol[o] = kEll16Pad;
            evals[o] = (V)0;
        }
    }
    if (bad) atomicOr(overflow, 1);
}

// Entries whose column equals that of the entry one row down and one slot
// to the left, (i, s) against (i+1, s-1), among the first w slots of each
// row (the ELL part of HYB; w >= the longest row for ELL): the x values an
// ELL product with neighbour reuse takes from a neighbouring row instead of
// gathering.  Integer sums (one atomic per workgroup), so the count is exact.
__global__ __launch_bounds__(kWG) void k_ell_reuse_count(int64_t n, const int *__restrict__ rp,
                                                         const int *__restrict__ col, int w,
                                                         unsigned long long *count) {
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    unsigned long long h = 0;
    if (i + 1 < n) {
        const int a0 = rp[i], la = min(rp[i + 1] - a0, w);
        const int b0 = rp[i + 1], lb = min(rp[i + 2] - b0, w);
        for (int s = 1; s < la && s - 1 < lb; ++s) h += col[a0 + s] == col[b0 + s - 1];
    }
    __shared__ unsigned long long sh[kWG / kWave];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) h += __shfl_xor(h, off, kWave);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = h;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int j = 0; j < kWG / kWave; ++j) t += sh[j];
        if (t) atomicAdd(count, t);
    }
}

template <typename V>
__global__ void k_csr_to_ell(int64_t n, int64_t n_pad, int w, const int *__restrict__ rp,
                             const int *__restrict__ col, const V *__restrict__ val,
                             int *__restrict__ ecol, V *__restrict__ evals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    int k0 = 0, len = 0;
    if (i < n) { k0 = rp[i]; len = rp[i + 1] - k0; }
    for (int s = 0; s < w; ++s) {
        int64_t o = (int64_t)s * n_pad + i;
        if (s < len) { ecol[o] = col[k0 + s]; evals[o] = val[k0 + s]; }
        else { ecol[o] = -1; evals[o] = (V)0; }
    }
}

template <typename V>
__global__ void k_hyb_tail(int64_t n, int k, const int *__restrict__ rp,
                           const int *__restrict__ col, const V *__restrict__ val,
                           const int64_t *__restrict__ toff, int *__restrict__ trow,
                           int *__restrict__ tcol, V *__restrict__ tval) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t t = toff[i];
    for (int e = rp[i] + k; e < rp[i + 1]; ++e, ++t) {
        trow[t] = (int)i;
        tcol[t] = col[e];
        tval[t] = val[e];
    }
}

// Column window of every 256-row tile (columns are sorted within rows, so
// the first and last entry of each row bound it).  Empty tile: lo > hi.
__global__ void k_ell_windows(int64_t n, const int *__restrict__ rp, const int *__restrict__ col,
                              int64_t ntiles, int tile_rows, int2 *__restrict__ win) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int lo = INT_MAX, hi = -1;
    int64_t r1 = (t + 1) * tile_rows < n ? (t + 1) * tile_rows : n;
    for (int64_t r = t * tile_rows; r < r1; ++r) {
        int a = rp[r], b = rp[r + 1];
        if (b > a) {
            lo = col[a] < lo ? col[a] : lo;
            hi = col[b - 1] > hi ? col[b - 1] : hi;
        }
    }
    if (hi < 0) lo = 0;
    win[t] = make_int2(lo, hi);
}

// Canonical-form check; sets bits of *flags: 1 start, 2 monotone, 4 end,
// 8 column range, 16 column order.
__global__ void k_validate(int64_t n, int64_t ncols, int64_t nnz, const int *__restrict__ rp,
                           const int *__restrict__ col, int *__restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (rp[0] != 0) atomicOr(flags, 1);
        if ((int64_t)rp[n] != nnz) atomicOr(flags, 4);
    }
    if (i >= n) return;
    int a = rp[i], b = rp[i + 1];
    if (b < a) { atomicOr(flags, 2); return; }
    if (a < 0 || (int64_t)b > nnz) { atomicOr(flags, 4); return; }
    int f = 0;
    for (int k = a; k < b; ++k) {
        int c = col[k];
        if (c < 0 || (int64_t)c >= ncols) f |= 8;
        if (k > a && c <= col[k - 1]) f |= 16;
    }
    if (f) atomicOr(flags, f);
}

// dinv_i = 1/a_ii in FP64, rounded to V.  *bad = smallest row with a missing
// or zero diagonal (initialised to INT_MAX by the host).
template <typename V>
__global__ void k_jacobi(int64_t n, const int *__restrict__ rp, const int *__restrict__ col,
                         const V *__restrict__ val, V *__restrict__ dinv, int *__restrict__ bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = rp[i], hi = rp[i + 1];
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (col[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    if (lo < rp[i + 1] && col[lo] == i && val[lo] != (V)0) {
        dinv[i] = (V)(1.0 / (double)val[lo]);
    } else {
        dinv[i] = (V)0;
        atomicMin(bad, (int)i);
    }
}

template <typename A, typename B>
__global__ void k_convert_vals(int64_t n, const A *__restrict__ in, B *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (B)in[i];
}

// ============================================================ host side

static int grid_for(int64_t tiles, int cap) {
    if (tiles <= 0) return 0;
    return (int)(tiles < cap ? tiles : cap);
}

int spmv_grid_cap(const MatrixImpl &A) {
    return A.ctx->num_cu * 8 < kMaxGrid ? A.ctx->num_cu * 8 : kMaxGrid;
}

// Plain applies (no fused dot) of the one-thread-per-row kernels run with up
// to 4x more workgroups: the band walk then keeps more rows in flight per XCD.
static int plain_grid(const MatrixImpl &A, int64_t tiles) {
    const int cap = 4 * spmv_grid_cap(A);
    return (int)(tiles < cap ? (tiles > 0 ? tiles : 1) : cap);
}

constexpr int kDotSlotCap = 8192;  // partial slots a fused-dot launch may publish

// Grids of the wave-walker kernels (4 walking waves per workgroup): a
// multiple of 8 workgroups keeps each walker on its XCD's band.
static int walker_grid(int64_t units, int cap) {
    if (units <= 0) return 0;  // nothing to launch (and no partial slots)
    int64_t g = (units + kWG / kWave - 1) / (kWG / kWave);
    g = g < cap ? g : cap;
    if (g >= kNumXcd) g -= g % kNumXcd;
    return (int)g;
}

// Points per thread of the matrix-free stencil: two consecutive points of
// an x-line when nx is even (128^3 27-point product 39.9 -> 26.8 us; four
// points hold 181 registers and take 30.6 us), else one.
static int stencil_rpt(const MatrixImpl &A) { return A.nx % 2 == 0 ? 2 : 1; }

void spmv_plan(MatrixImpl &A) {
    const int cap = spmv_grid_cap(A);
    A.grid_main = A.grid_tail = 0;
    A.grid_dot = 0;
    switch (A.format) {
    case MXL_FMT_CSR:
        if (A.variant == MXL_CSR_SCALAR) A.grid_main = grid_for((A.nrows + kWG - 1) / kWG, cap);
        else if (A.variant == MXL_CSR_VECTOR)
            A.grid_main = grid_for((A.nrows + kWG / A.vw - 1) / (kWG / A.vw), cap);
        else if (A.variant == MXL_CSR_STREAM) A.grid_main = walker_grid(A.ntiles, cap);
        else A.grid_main = grid_for(A.ntiles, cap);
        break;
    case MXL_FMT_COO:
        A.grid_main = walker_grid(A.ntiles, cap);
        break;
    case MXL_FMT_STENCIL:
        A.grid_main = grid_for((A.nrows + (int64_t)kWG * stencil_rpt(A) - 1) / ((int64_t)kWG * stencil_rpt(A)), cap);
        break;
    case MXL_FMT_ELL: {
        const int64_t tiles = (A.nrows + kWG * A.ell_rpt - 1) / (kWG * A.ell_rpt);
        A.grid_main = grid_for(tiles, cap);
        // fused-dot launches: one tile per workgroup while the partials fit
        A.grid_dot = tiles <= kDotSlotCap ? (int)(tiles > 0 ? tiles : 1) : A.grid_main;
        break;
    }
    case MXL_FMT_HYB:
        A.grid_main = grid_for((A.nrows + kWG * A.ell_rpt - 1) / (kWG * A.ell_rpt), cap);
        A.grid_dot = A.grid_main;  // the tail's partials follow the ELL part's
        A.grid_tail = walker_grid(A.ntiles, cap);
        break;
    }
}

int spmv_slots(const MatrixImpl &A) {
    return (A.format == MXL_FMT_ELL ? A.grid_dot : A.grid_main) + A.grid_tail;
}

void stream_blocks(const std::vector<int32_t> &rp, std::vector<int32_t> &out) {
    const int64_t n = (int64_t)rp.size() - 1;
    out.clear();
    int64_t r = 0;
    while (r < n) {
        out.push_back((int32_t)r);
        out.push_back(rp[r]);
        int64_t r1 = r + 1;
        if (rp[r + 1] - rp[r] <= kStreamK * kWave)
            while (r1 < n && r1 - r < kStreamRows && rp[r1 + 1] - rp[r] <= kStreamK * kWave) ++r1;
        r = r1;
    }
    out.push_back((int32_t)n);
    out.push_back(n >= 0 ? rp[n] : 0);
}

int64_t merge_tiles(int64_t n, int64_t nnz) { return (n + nnz + kMergeItems - 1) / kMergeItems; }
int64_t coo_tiles(int64_t nnz) { return (nnz + kCooWaveItems - 1) / kCooWaveItems; }
int64_t carry_bytes(int64_t ntiles) { return (ntiles > 0 ? ntiles : 1) * (int64_t)sizeof(Carry); }
int ell_lds_cap() { return kEllLdsCap; }

hipError_t merge_partition(const MatrixImpl &A, hipStream_t s) {
    int64_t nb = A.ntiles + 1;
    int g = (int)((nb + 255) / 256);
    hipLaunchKernelGGL(k_merge_partition, dim3(g), dim3(256), 0, s, A.nrows, A.nnz,
                       (const int *)A.row_ptr->p, A.ntiles, (int2 *)A.part->p);
    return hipGetLastError();
}

template <typename V>
static hipError_t spmv_typed(const MatrixImpl &A, const SpmvArgs &a, hipStream_t s) {
    SpmvK<V> p;
    p.x = (const V *)a.x;
    p.y = (V *)a.y;
    p.alpha = (V)a.alpha;
    p.beta = (V)a.beta;
    p.beta_zero = (a.beta == 0.0);
    p.stop = a.stop;
    p.w = (const V *)a.w;
    p.partials = a.partials;
    p.slot_base = 0;
    const bool dot = a.w != nullptr;
    const int64_t n = A.nrows;
    if (n == 0) return hipSuccess;
    // a matrix-free stencil has no arrays
    const int *rp = A.row_ptr ? (const int *)A.row_ptr->p : nullptr;
    const int *col = A.col ? (const int *)A.col->p : nullptr;
    const V *val = A.val ? (const V *)A.val->p : nullptr;
    const dim3 blk(kWG);
    auto fixup = [&](const Carry *cr, int64_t ntiles) {
        const unsigned g = (unsigned)((ntiles + kWG - 1) / kWG);
        if (g) hipLaunchKernelGGL(k_carry_fixup<V>, dim3(g), blk, 0, s, cr, ntiles, p);
    };
    switch (A.format) {
    case MXL_FMT_CSR: {
        if (A.variant == MXL_CSR_SCALAR) {
            if (dot) hipLaunchKernelGGL((k_csr_scalar<V, true>), dim3(A.grid_main), blk, 0, s, n, rp, col, val, p);
            else hipLaunchKernelGGL((k_csr_scalar<V, false>), dim3(A.grid_main), blk, 0, s, n, rp, col, val, p);
        } else if (A.variant == MXL_CSR_VECTOR) {
#define MXL_VEC_CASE(WW)                                                                                   \
    case WW:                                                                                               \
        if (dot) hipLaunchKernelGGL((k_csr_vector<V, WW, true>), dim3(A.grid_main), blk, 0, s, n, rp, col, val, p); \
        else hipLaunchKernelGGL((k_csr_vector<V, WW, false>), dim3(A.grid_main), blk, 0, s, n, rp, col, val, p); \
        break;
            switch (A.vw) {
                MXL_VEC_CASE(2) MXL_VEC_CASE(4) MXL_VEC_CASE(8) MXL_VEC_CASE(16) MXL_VEC_CASE(32) MXL_VEC_CASE(64)
            default: return hipErrorInvalidValue;
            }
#undef MXL_VEC_CASE
        } else if (A.variant == MXL_CSR_STREAM) {
            const int2 *bk = (const int2 *)A.part->p;
            if (dot) hipLaunchKernelGGL((k_csr_stream<V, true>), dim3(A.grid_main), blk, 0, s, A.ntiles, bk, rp, col, val, p);
            else hipLaunchKernelGGL((k_csr_stream<V, false>), dim3(A.grid_main), blk, 0, s, A.ntiles, bk, rp, col, val, p);
        } else {
            Carry *cr = (Carry *)A.carries->p;
            const int2 *part = (const int2 *)A.part->p;
            if (dot) hipLaunchKernelGGL((k_csr_merge<V, true>), dim3(A.grid_main), blk, 0, s, n, rp, col, val, part, A.ntiles, cr, p);
            else hipLaunchKernelGGL((k_csr_merge<V, false>), dim3(A.grid_main), blk, 0, s, n, rp, col, val, part, A.ntiles, cr, p);
            fixup(cr, A.ntiles);
        }
        break;
    }
    case MXL_FMT_STENCIL: {
        StencilK sk{};
        sk.nx = (int)A.nx;
        sk.ny = (int)A.ny;
        sk.nz = (int)A.nz;
        sk.inv_nx = 1.0 / (double)A.nx;
        sk.inv_nxy = 1.0 / ((double)A.nx * (double)A.ny);
        bool star = true;
        for (int q = 0; q < A.st_npts; ++q) {
            const int di = A.st_off[q][0], dj = A.st_off[q][1], dk = A.st_off[q][2];
            const int c = 9 * (dk + 1) + 3 * (dj + 1) + (di + 1);
            sk.mask |= 1u << c;
            sk.c[c] = A.st_coef[q];
            star = star && (di != 0) + (dj != 0) + (dk != 0) <= 1;
        }
        const dim3 g(A.grid_main);
#define MXL_ST_CASE(RR)                                                                           \
    case RR:                                                                                      \
        if (star) {                                                                               \
            if (dot) hipLaunchKernelGGL((k_stencil<V, true, true, RR>), g, blk, 0, s, sk, p);     \
            else hipLaunchKernelGGL((k_stencil<V, false, true, RR>), g, blk, 0, s, sk, p);        \
        } else {                                                                                  \
            if (dot) hipLaunchKernelGGL((k_stencil<V, true, false, RR>), g, blk, 0, s, sk, p);    \
            else hipLaunchKernelGGL((k_stencil<V, false, false, RR>), g, blk, 0, s, sk, p);       \
        }                                                                                         \
        break;
        switch (stencil_rpt(A)) {
            MXL_ST_CASE(1) MXL_ST_CASE(2)
        default: return hipErrorInvalidValue;
        }
#undef MXL_ST_CASE
        break;
    }
    case MXL_FMT_COO: {
        if (A.nnz == 0) {
            if (dot) return hipErrorNotSupported;
            hipLaunchKernelGGL(k_scale_only<V>, dim3(256), blk, 0, s, n, p);
            break;
        }
        Carry *cr = (Carry *)A.carries->p;
        const int *row = (const int *)A.coo_row->p;
        if (dot) hipLaunchKernelGGL((k_coo_wave<V, true, false>), dim3(A.grid_main), blk, 0, s, n, A.nnz, row, col, val, A.ntiles, cr, p);
        else hipLaunchKernelGGL((k_coo_wave<V, false, false>), dim3(A.grid_main), blk, 0, s, n, A.nnz, row, col, val, A.ntiles, cr, p);
        fixup(cr, A.ntiles);
        break;
    }
    case MXL_FMT_ELL:
    case MXL_FMT_HYB: {
        const void *ec = A.ell_col->p;
        const V *ev = (const V *)A.ell_val->p;
        const int2 *win = A.ell_win ? (const int2 *)A.ell_win->p : nullptr;
        const bool lds = A.variant == MXL_ELL_LDS && win;
        const bool d16 = A.format == MXL_FMT_ELL && A.variant == MXL_ELL_DELTA16;
        const bool nb = A.ell_nb && !lds;  // ELL or the ELL part of HYB
        const dim3 ge(dot ? A.grid_dot
                          : plain_grid(A, (n + (int64_t)kWG * A.ell_rpt - 1) / ((int64_t)kWG * A.ell_rpt)));
#define MXL_ELL_CASE(RR)                                                                                          \
    case RR:                                                                                                      \
        if (d16 && nb) {                                                                                          \
            if (dot) hipLaunchKernelGGL((k_ell<V, true, false, RR, true, true>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p); \
            else hipLaunchKernelGGL((k_ell<V, false, false, RR, true, true>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p);    \
        } else if (d16) {                                                                                         \
            if (dot) hipLaunchKernelGGL((k_ell<V, true, false, RR, true>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p); \
            else hipLaunchKernelGGL((k_ell<V, false, false, RR, true>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p);    \
        } else if (lds) {                                                                                         \
            if (dot) hipLaunchKernelGGL((k_ell<V, true, true, RR>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p);   \
            else hipLaunchKernelGGL((k_ell<V, false, true, RR>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p);      \
        } else if (nb) {                                                                                          \
            if (dot) hipLaunchKernelGGL((k_ell<V, true, false, RR, false, true>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p); \
            else hipLaunchKernelGGL((k_ell<V, false, false, RR, false, true>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p);    \
        } else {                                                                                                  \
            if (dot) hipLaunchKernelGGL((k_ell<V, true, false, RR>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p);  \
            else hipLaunchKernelGGL((k_ell<V, false, false, RR>), ge, blk, 0, s, n, A.n_pad, A.ell_w, ec, ev, win, p);     \
        }                                                                                                         \
        break;
        switch (A.ell_rpt) {
            MXL_ELL_CASE(1) MXL_ELL_CASE(2) MXL_ELL_CASE(4)
        default: return hipErrorInvalidValue;
        }
#undef MXL_ELL_CASE
        if (A.format == MXL_FMT_HYB && A.tail_nnz > 0) {
            SpmvK<V> t = p;  // tail accumulates into y
            t.slot_base = A.grid_main;
            t.beta = (V)1;
            t.beta_zero = 0;
            Carry *cr = (Carry *)A.carries->p;
            const int *tr = (const int *)A.tail_row->p;
            const int *tc = (const int *)A.tail_col->p;
            const V *tv = (const V *)A.tail_val->p;
            if (dot) hipLaunchKernelGGL((k_coo_wave<V, true, true>), dim3(A.grid_tail), blk, 0, s, n, A.tail_nnz, tr, tc, tv, A.ntiles, cr, t);
            else hipLaunchKernelGGL((k_coo_wave<V, false, true>), dim3(A.grid_tail), blk, 0, s, n, A.tail_nnz, tr, tc, tv, A.ntiles, cr, t);
            fixup(cr, A.ntiles);
        }
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t spmv_launch(const MatrixImpl &A, const SpmvArgs &a, hipStream_t s) {
    return A.dtype == MXL_F64 ? spmv_typed<double>(A, a, s) : spmv_typed<float>(A, a, s);
}

// ---------------------------------------------------- setup launchers
static dim3 g1(int64_t n) { return dim3((unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1)); }

hipError_t launch_validate(const MatrixImpl &A, int *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, g1(A.nrows + 1), dim3(256), 0, s, A.nrows, A.ncols, A.nnz,
                       (const int *)A.row_ptr->p, (const int *)A.col->p, flags);
    return hipGetLastError();
}

hipError_t launch_csr_to_coo(const MatrixImpl &A, int *row, hipStream_t s) {
    if (A.nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_csr_to_coo, g1(A.nrows), dim3(256), 0, s, A.nrows, (const int *)A.row_ptr->p, row);
    return hipGetLastError();
}

hipError_t launch_csr_to_ell(const MatrixImpl &A, int w, int64_t n_pad, int *ecol, void *evals,
                             hipStream_t s) {
    if (n_pad == 0 || w == 0) return hipSuccess;
    if (A.dtype == MXL_F64)
        hipLaunchKernelGGL(k_csr_to_ell<double>, g1(n_pad), dim3(256), 0, s, A.nrows, n_pad, w,
                           (const int *)A.row_ptr->p, (const int *)A.col->p,
                           (const double *)A.val->p, ecol, (double *)evals);
    else
        hipLaunchKernelGGL(k_csr_to_ell<float>, g1(n_pad), dim3(256), 0, s, A.nrows, n_pad, w,
                           (const int *)A.row_ptr->p, (const int *)A.col->p,
                           (const float *)A.val->p, ecol, (float *)evals);
    return hipGetLastError();
}

hipError_t launch_csr_to_ell16(const MatrixImpl &A, int w, int64_t n_pad, short *ecol, void *evals,
                               int *overflow, hipStream_t s) {
    if (n_pad == 0 || w == 0) return hipSuccess;
    if (A.dtype == MXL_F64)
        hipLaunchKernelGGL(k_csr_to_ell16<double>, g1(n_pad), dim3(256), 0, s, A.nrows, n_pad, w,
                           (const int *)A.row_ptr->p, (const int *)A.col->p,
                           (const double *)A.val->p, ecol, (double *)evals, overflow);
    else
        hipLaunchKernelGGL(k_csr_to_ell16<float>, g1(n_pad), dim3(256), 0, s, A.nrows, n_pad, w,
                           (const int *)A.row_ptr->p, (const int *)A.col->p,
                           (const float *)A.val->p, ecol, (float *)evals, overflow);
    return hipGetLastError();
}

hipError_t launch_ell_reuse_count(const MatrixImpl &A, int w, unsigned long long *count, hipStream_t s) {
    if (A.nrows < 2) return hipSuccess;
    hipLaunchKernelGGL(k_ell_reuse_count, g1(A.nrows), dim3(kWG), 0, s, A.nrows, (const int *)A.row_ptr->p,
                       (const int *)A.col->p, w, count);
    return hipGetLastError();
}

hipError_t launch_hyb_tail(const MatrixImpl &A, int k, const int64_t *toff, int *trow, int *tcol,
                           void *tval, hipStream_t s) {
    if (A.nrows == 0) return hipSuccess;
    if (A.dtype == MXL_F64)
        hipLaunchKernelGGL(k_hyb_tail<double>, g1(A.nrows), dim3(256), 0, s, A.nrows, k,
                           (const int *)A.row_ptr->p, (const int *)A.col->p,
                           (const double *)A.val->p, toff, trow, tcol, (double *)tval);
    else
        hipLaunchKernelGGL(k_hyb_tail<float>, g1(A.nrows), dim3(256), 0, s, A.nrows, k,
                           (const int *)A.row_ptr->p, (const int *)A.col->p,
                           (const float *)A.val->p, toff, trow, tcol, (float *)tval);
    return hipGetLastError();
}

hipError_t launch_ell_windows(const MatrixImpl &A, int2 *win, hipStream_t s) {
    const int tr = kWG * A.ell_rpt;
    int64_t nt = (A.nrows + tr - 1) / tr;
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ell_windows, g1(nt), dim3(256), 0, s, A.nrows, (const int *)A.row_ptr->p,
                       (const int *)A.col->p, nt, tr, win);
    return hipGetLastError();
}

hipError_t launch_jacobi(const MatrixImpl &A, void *dinv, int *bad, hipStream_t s) {
    if (A.nrows == 0) return hipSuccess;
    if (A.dtype == MXL_F64)
        hipLaunchKernelGGL(k_jacobi<double>, g1(A.nrows), dim3(256), 0, s, A.nrows,
                           (const int *)A.row_ptr->p, (const int *)A.col->p,
                           (const double *)A.val->p, (double *)dinv, bad);
    else
        hipLaunchKernelGGL(k_jacobi<float>, g1(A.nrows), dim3(256), 0, s, A.nrows,
                           (const int *)A.row_ptr->p, (const int *)A.col->p,
                           (const float *)A.val->p, (float *)dinv, bad);
    return hipGetLastError();
}

hipError_t launch_convert_vals(int64_t n, int from, const void *in, void *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    unsigned g = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    if (from == MXL_F64)
        hipLaunchKernelGGL((k_convert_vals<double, float>), dim3(g), dim3(256), 0, s, n, (const double *)in, (float *)out);
    else
        hipLaunchKernelGGL((k_convert_vals<float, double>), dim3(g), dim3(256), 0, s, n, (const float *)in, (double *)out);
    return hipGetLastError();
}

}  // namespace mxl
