// select.hip -- the format/kernel selector's device work: the 16 structural
// features of a CSR matrix, and a small FP32 multilayer perceptron with its
// forward pass, gradient and Adam step, so the selector is trained on the
// GPU by this library's own kernels.  The selector stands in for the
// paper's runtime "kernel variant selection" fork (Sec. 7.2), and its quality
// is scored with the performance-profile view of Sec. 7.3.
//
// Features use exact integer statistics: sums of len, len^2, len^3, |i-j|,
// counts and extrema are accumulated as 64-bit integers (order-independent,
// hence deterministic); quantiles come from a row-length histogram.  The
// host turns the exact integers into the 16 FP64 values.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "internal.hpp"

namespace mxl {

struct FeatAcc {
    unsigned long long s2, s3, above, sumbw, near;
    int maxlen, minlen, maxbw, pad;
};

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
    return v;
}

// Row statistics: thread per row (grid-stride).  Row lengths below
// kHistBins are counted in a per-workgroup LDS histogram that is added to
// the global one bin by bin at the end (rows of equal length would
// otherwise serialise on one global counter); the sums, minima and maxima
// are reduced over the workgroup and combined with one integer atomic each
// (exact, so the order does not matter).
constexpr int kHistBins = 4096;

__global__ __launch_bounds__(kWG) void k_features(int64_t n, int64_t nnz, const int *__restrict__ rp,
                                                  const int *__restrict__ col,
                                                  FeatAcc *__restrict__ acc,
                                                  unsigned *__restrict__ hist, int maxlen_all) {
    constexpr int NW = kWG / kWave;
    __shared__ unsigned sh[kHistBins];
    __shared__ unsigned long long s_u[5][NW];
    __shared__ int s_i[3][NW];
    const int nbins = maxlen_all + 1 < kHistBins ? maxlen_all + 1 : kHistBins;
    for (int j = threadIdx.x; j < nbins; j += kWG) sh[j] = 0u;
    __syncthreads();
    unsigned long long s2 = 0, s3 = 0, above = 0, sumbw = 0, near = 0;
    int maxlen = 0, minlen = INT_MAX, maxbw = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int a = rp[i], b = rp[i + 1];
        const unsigned long long len = (unsigned long long)(b - a);
        s2 += len * len;
        s3 += len * len * len;
        if ((int64_t)len * n > 2 * nnz) ++above;
        maxlen = max(maxlen, (int)len);
        minlen = min(minlen, (int)len);
        if (len < (unsigned long long)kHistBins) atomicAdd(&sh[len], 1u);
        else atomicAdd(hist + len, 1u);
        for (int e = a; e < b; ++e) {
            long long d = (long long)col[e] - i;
            d = d < 0 ? -d : d;
            sumbw += (unsigned long long)d;
            near += d <= 64;
            maxbw = max(maxbw, (int)d);
        }
    }
    s2 = wave_sum_u64(s2);
    s3 = wave_sum_u64(s3);
    above = wave_sum_u64(above);
    sumbw = wave_sum_u64(sumbw);
    near = wave_sum_u64(near);
    maxlen = wave_max_i(maxlen);
    minlen = wave_min_i(minlen);
    maxbw = wave_max_i(maxbw);
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
        s_u[0][w] = s2;
        s_u[1][w] = s3;
        s_u[2][w] = above;
        s_u[3][w] = sumbw;
        s_u[4][w] = near;
        s_i[0][w] = maxlen;
        s_i[1][w] = minlen;
        s_i[2][w] = maxbw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < NW; ++v) {
            s2 += s_u[0][v];
            s3 += s_u[1][v];
            above += s_u[2][v];
            sumbw += s_u[3][v];
            near += s_u[4][v];
            maxlen = max(maxlen, s_i[0][v]);
            minlen = min(minlen, s_i[1][v]);
            maxbw = max(maxbw, s_i[2][v]);
        }
        atomicAdd(&acc->s2, s2);
        atomicAdd(&acc->s3, s3);
        atomicAdd(&acc->above, above);
        atomicAdd(&acc->sumbw, sumbw);
        atomicAdd(&acc->near, near);
        atomicMax(&acc->maxlen, maxlen);
        atomicMin(&acc->minlen, minlen);
        atomicMax(&acc->maxbw, maxbw);
    }
    for (int j = threadIdx.x; j < nbins; j += kWG)
        if (sh[j]) atomicAdd(hist + j, sh[j]);
}

__global__ void k_row_maxlen(int64_t n, const int *__restrict__ rp, int *__restrict__ out) {
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, rp[i + 1] - rp[i]);
    m = wave_max_i(m);
    if (threadIdx.x % kWave == 0) atomicMax(out, m);
}

// ------------------------------------------------------------------ MLP
// Layer l maps dims[l] -> dims[l+1]; theta packs W_l (row-major) then b_l.
// One workgroup per sample runs the forward pass and back-propagation in
// LDS and writes that sample's gradient contribution; a second kernel sums
// the contributions over samples in index order (deterministic) and adds
// the weight-decay term.  Widths are at most kMlpMaxW.
constexpr int kMlpMaxW = 64;
constexpr int kMlpMaxL = 6;

struct MlpShape {
    int nl;
    int dims[kMlpMaxL + 1];
    int off[kMlpMaxL];  // parameter offset of W_l
    int nparams;
};

__global__ __launch_bounds__(kWave) void k_mlp_sample(MlpShape sh, const float *__restrict__ theta,
                                                      const float *__restrict__ X,
                                                      const float *__restrict__ T,
                                                      const float *__restrict__ M, float inv_msum,
                                                      float *__restrict__ Y, float *__restrict__ gs,
                                                      float *__restrict__ loss_s, int want_grad) {
    __shared__ float act[kMlpMaxL + 1][kMlpMaxW];  // activations a_0..a_L
    __shared__ float pre[kMlpMaxL + 1][kMlpMaxW];  // pre-activations h_1..h_L
    __shared__ float dh[2][kMlpMaxW];
    const int smp = blockIdx.x, t = threadIdx.x;
    const int L = sh.nl;
    if (t < sh.dims[0]) act[0][t] = X[(int64_t)smp * sh.dims[0] + t];
    __syncthreads();
    for (int l = 0; l < L; ++l) {
        const int din = sh.dims[l], dout = sh.dims[l + 1];
        const float *W = theta + sh.off[l];
        const float *bb = W + dout * din;
        if (t < dout) {
            float a = bb[t];
            for (int j = 0; j < din; ++j) a += W[t * din + j] * act[l][j];
            pre[l + 1][t] = a;
            act[l + 1][t] = (l < L - 1) ? fmaxf(a, 0.f) : a;
        }
        __syncthreads();
    }
    const int C = sh.dims[L];
    float le = 0.f;
    if (t < C) {
        const float yv = act[L][t];
        if (Y) Y[(int64_t)smp * C + t] = yv;
        if (T) {
            const float e = yv - T[(int64_t)smp * C + t];
            const float m = M[(int64_t)smp * C + t];
            le = m * e * e;
            dh[L & 1][t] = 2.f * m * e * inv_msum;
        }
    }
    if (loss_s) {
        float v = le;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
        if (t == 0) loss_s[smp] = v;
    }
    if (!want_grad) return;
    __syncthreads();
    float *g = gs + (int64_t)smp * sh.nparams;
    for (int l = L - 1; l >= 0; --l) {
        const int din = sh.dims[l], dout = sh.dims[l + 1];
        const float *W = theta + sh.off[l];
        float *gW = g + sh.off[l];
        float *gb = gW + dout * din;
        const float *d = dh[(l + 1) & 1];
        for (int idx = t; idx < dout * din; idx += kWave) gW[idx] = d[idx / din] * act[l][idx % din];
        if (t < dout) gb[t] = d[t];
        if (l > 0 && t < din) {
            float a = 0.f;
            for (int o = 0; o < dout; ++o) a += W[o * din + t] * d[o];
            dh[l & 1][t] = pre[l][t] > 0.f ? a : 0.f;
        }
        __syncthreads();
    }
}

__global__ void k_mlp_reduce(MlpShape sh, int64_t nsamples, const float *__restrict__ theta,
                             const float *__restrict__ gs, float lambda, float *__restrict__ grad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= sh.nparams) return;
    float s = 0.f;
    for (int64_t k = 0; k < nsamples; ++k) s += gs[k * sh.nparams + j];
    // weight decay on W entries only
    bool is_w = false;
    for (int l = 0; l < sh.nl; ++l) {
        const int w0 = sh.off[l], w1 = w0 + sh.dims[l] * sh.dims[l + 1];
        if (j >= w0 && j < w1) is_w = true;
    }
    grad[j] = s + (is_w ? 2.f * lambda * theta[j] : 0.f);
}

__global__ void k_adam(int n, float *__restrict__ theta, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.f - b1) * gj;
    const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    theta[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

}  // namespace mxl

using namespace mxl;

// ================================================================== host
namespace mxl {

mxl_status features_compute(const MatrixImpl &A, double out[16], std::vector<unsigned> *hist_out,
                            int64_t *maxbw_out) {
    mxl_ctx *ctx = A.ctx;
    hipStream_t s = ctx->stream;
    for (int j = 0; j < 16; ++j) out[j] = 0.0;
    const int64_t n = A.nrows, nnz = A.nnz;
    if (n == 0) return MXL_OK;
    void *dmax = nullptr, *dacc = nullptr, *dhist = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(dmax);
        (void)hipFree(dacc);
        (void)hipFree(dhist);
    };
    if (hipMalloc(&dmax, 4) != hipSuccess || hipMalloc(&dacc, sizeof(FeatAcc)) != hipSuccess) {
        cleanup();
        return set_error(MXL_ERR_OUT_OF_MEMORY, "features workspace");
    }
    const unsigned G = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    int zero = 0;
    FeatAcc init{};
    init.minlen = INT_MAX;
    if (hipMemcpyAsync(dmax, &zero, 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(dacc, &init, sizeof init, hipMemcpyHostToDevice, s) != hipSuccess) {
        cleanup();
        return set_error(MXL_ERR_DEVICE, "features init");
    }
    hipLaunchKernelGGL(k_row_maxlen, dim3(G), dim3(256), 0, s, n, (const int *)A.row_ptr->p, (int *)dmax);
    int maxlen = 0;
    if (hipMemcpyAsync(&maxlen, dmax, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        cleanup();
        return set_error(MXL_ERR_DEVICE, "features max length");
    }
    if (hipMalloc(&dhist, (size_t)(maxlen + 1) * 4) != hipSuccess ||
        hipMemsetAsync(dhist, 0, (size_t)(maxlen + 1) * 4, s) != hipSuccess) {
        cleanup();
        return set_error(MXL_ERR_OUT_OF_MEMORY, "features histogram");
    }
    const unsigned Gf = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_features, dim3(Gf), dim3(kWG), 0, s, n, nnz, (const int *)A.row_ptr->p,
                       (const int *)A.col->p, (FeatAcc *)dacc, (unsigned *)dhist, maxlen);
    FeatAcc h;
    std::vector<unsigned> hist((size_t)maxlen + 1);
    if (hipMemcpyAsync(&h, dacc, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hist.data(), dhist, hist.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        cleanup();
        return set_error(MXL_ERR_DEVICE, "features read-back");
    }
    cleanup();
    if (hist_out) *hist_out = hist;
    if (maxbw_out) *maxbw_out = (int64_t)h.maxbw;
    // nearest-rank quantiles: sorted length at 1-based rank ceil(P*n/100)
    auto quant = [&](int P) {
        const int64_t rank = (P * n + 99) / 100;
        int64_t cum = 0;
        for (size_t L = 0; L < hist.size(); ++L) {
            cum += hist[L];
            if (cum >= rank) return (double)L;
        }
        return (double)maxlen;
    };
    typedef __int128 i128;
    const double dn = (double)n;
    const i128 S1 = nnz, S2 = (i128)h.s2, S3 = (i128)h.s3, N = n;
    const double m2 = (double)(N * S2 - S1 * S1) / (dn * dn);                       // population variance
    const double m3 = (double)(N * N * S3 - 3 * N * S1 * S2 + 2 * S1 * S1 * S1) / (dn * dn * dn);
    const double mu = (double)nnz / dn;
    const double sigma = std::sqrt(std::max(m2, 0.0));
    out[0] = std::log10(dn);
    out[1] = std::log10(nnz > 0 ? (double)nnz : 1.0);
    out[2] = mu;
    out[3] = sigma;
    out[4] = mu > 0.0 ? sigma / mu : 0.0;
    out[5] = (double)h.maxlen;
    out[6] = (double)h.minlen;
    out[7] = quant(50);
    out[8] = quant(90);
    out[9] = quant(99);
    out[10] = (double)h.above / dn;
    out[11] = nnz > 0 ? dn * (double)h.maxlen / (double)nnz : 0.0;
    out[12] = (double)h.maxbw / dn;
    out[13] = nnz > 0 ? (double)h.sumbw / (double)nnz / dn : 0.0;
    out[14] = nnz > 0 ? (double)h.near / (double)nnz : 0.0;
    out[15] = m2 > 0.0 ? m3 / std::pow(m2, 1.5) : 0.0;
    return MXL_OK;
}

}  // namespace mxl

struct mxl_mlp {
    CtxRef ctx;
    MlpShape sh{};
    void *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    void *gs = nullptr;  // per-sample gradients
    int64_t gs_cap = 0;
    float loss = 0.f;
};

extern "C" mxl_status mxl_features(const mxl_op *Aop, double out_host[16]) try {
    if (!Aop || Aop->kind != MXL_OP_MATRIX || !out_host)
        return set_error(MXL_ERR_INVALID_ARG, "matrix operator and output required");
    if (Aop->mat->format == MXL_FMT_STENCIL)
        return set_error(MXL_ERR_NOT_IMPLEMENTED, "a matrix-free stencil has no rows to describe");
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(Aop->mat->ctx->device);
    mxl_status st = features_compute(*Aop->mat, out_host);
    if (prev >= 0) (void)hipSetDevice(prev);
    return st;
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_mlp_create(mxl_ctx *ctx, int32_t nlayers, const int32_t *dims,
                                     const float *theta_host, mxl_mlp **out) try {
    if (!ctx || !dims || !out || nlayers < 1 || nlayers > kMlpMaxL)
        return set_error(MXL_ERR_INVALID_ARG, "mlp: 1..6 layers, dims and out required");
    *out = nullptr;
    MlpShape sh{};
    sh.nl = nlayers;
    int off = 0;
    for (int l = 0; l <= nlayers; ++l) {
        if (dims[l] < 1 || dims[l] > kMlpMaxW) return set_error(MXL_ERR_INVALID_ARG, "mlp widths must be 1..64");
        sh.dims[l] = dims[l];
    }
    for (int l = 0; l < nlayers; ++l) {
        sh.off[l] = off;
        off += dims[l + 1] * dims[l] + dims[l + 1];
    }
    sh.nparams = off;
    auto *mm = new mxl_mlp;
    mm->ctx = ctx;
    mm->sh = sh;
    const size_t pb = (size_t)off * 4;
    if (hipMalloc(&mm->theta, pb) != hipSuccess || hipMalloc(&mm->grad, pb) != hipSuccess ||
        hipMalloc(&mm->m, pb) != hipSuccess || hipMalloc(&mm->v, pb) != hipSuccess) {
        mxl_mlp_destroy(mm);
        return set_error(MXL_ERR_OUT_OF_MEMORY, "mlp parameters");
    }
    hipStream_t s = ctx->stream;
    std::vector<float> zeros(off, 0.f);
    if ((theta_host && hipMemcpyAsync(mm->theta, theta_host, pb, hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipMemcpyAsync(mm->grad, zeros.data(), pb, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(mm->m, zeros.data(), pb, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(mm->v, zeros.data(), pb, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        mxl_mlp_destroy(mm);
        return set_error(MXL_ERR_DEVICE, "mlp upload");
    }
    *out = mm;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

static mxl_status mlp_copy(const mxl_mlp *mm, void *dst, const void *src, int64_t n, hipMemcpyKind k) {
    if (!mm || !dst || !src || n != mm->sh.nparams)
        return set_error(MXL_ERR_DIM_MISMATCH, "parameter count does not match the network");
    if (hipMemcpyAsync(dst, src, (size_t)n * 4, k, mm->ctx->stream) != hipSuccess ||
        hipStreamSynchronize(mm->ctx->stream) != hipSuccess)
        return set_error(MXL_ERR_DEVICE, "mlp copy");
    return MXL_OK;
}

extern "C" mxl_status mxl_mlp_get_params(const mxl_mlp *mm, float *theta_host, int64_t n) try {
    return mlp_copy(mm, theta_host, mm ? mm->theta : nullptr, n, hipMemcpyDeviceToHost);
} catch (...) {
    return mxl::abi_exception(__func__);
}
extern "C" mxl_status mxl_mlp_set_params(mxl_mlp *mm, const float *theta_host, int64_t n) try {
    return mlp_copy(mm, mm ? mm->theta : nullptr, theta_host, n, hipMemcpyHostToDevice);
} catch (...) {
    return mxl::abi_exception(__func__);
}
extern "C" mxl_status mxl_mlp_get_grad(const mxl_mlp *mm, float *grad_host, int64_t n) try {
    return mlp_copy(mm, grad_host, mm ? mm->grad : nullptr, n, hipMemcpyDeviceToHost);
} catch (...) {
    return mxl::abi_exception(__func__);
}

static mxl_status mlp_run(mxl_mlp *mm, int64_t ns, const float *X, const float *T, const float *M,
                          float lambda, float *Y, float *loss_host, bool grad) {
    if (!mm || ns < 1 || !X) return set_error(MXL_ERR_INVALID_ARG, "mlp: network, samples >= 1, X");
    mxl_status st;
    const int C = mm->sh.dims[mm->sh.nl];
    if ((st = check_device_ptr(mm->ctx, X, (size_t)ns * mm->sh.dims[0] * 4, "X")) != MXL_OK) return st;
    if (Y && (st = check_device_ptr(mm->ctx, Y, (size_t)ns * C * 4, "Y")) != MXL_OK) return st;
    hipStream_t s = mm->ctx->stream;
    float inv = 0.f;
    void *lossd = nullptr;
    if (T) {
        if ((st = check_device_ptr(mm->ctx, T, (size_t)ns * C * 4, "T")) != MXL_OK) return st;
        if ((st = check_device_ptr(mm->ctx, M, (size_t)ns * C * 4, "M")) != MXL_OK) return st;
        std::vector<float> mh((size_t)ns * C);
        if (hipMemcpyAsync(mh.data(), M, mh.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return set_error(MXL_ERR_DEVICE, "mask read");
        double msum = 0.0;
        for (float v : mh) msum += v;
        inv = msum > 0 ? (float)(1.0 / msum) : 0.f;
        if (hipMalloc(&lossd, (size_t)ns * 4) != hipSuccess) return set_error(MXL_ERR_OUT_OF_MEMORY, "loss");
    }
    if (grad && mm->gs_cap < ns) {
        (void)hipFree(mm->gs);
        mm->gs = nullptr;
        if (hipMalloc(&mm->gs, (size_t)ns * mm->sh.nparams * 4) != hipSuccess) {
            (void)hipFree(lossd);
            mm->gs_cap = 0;
            return set_error(MXL_ERR_OUT_OF_MEMORY, "per-sample gradients");
        }
        mm->gs_cap = ns;
    }
    hipLaunchKernelGGL(k_mlp_sample, dim3((unsigned)ns), dim3(kWave), 0, s, mm->sh, (const float *)mm->theta,
                       X, T, M, inv, Y, (float *)mm->gs, (float *)lossd, grad ? 1 : 0);
    if (grad)
        hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((mm->sh.nparams + 255) / 256)), dim3(256), 0, s,
                           mm->sh, ns, (const float *)mm->theta, (const float *)mm->gs, lambda,
                           (float *)mm->grad);
    if (hipGetLastError() != hipSuccess) {
        (void)hipFree(lossd);
        return set_error(MXL_ERR_DEVICE, "mlp launch");
    }
    if (T) {
        std::vector<float> lh(ns);
        std::vector<float> th(mm->sh.nparams);
        hipError_t e = hipMemcpyAsync(lh.data(), lossd, (size_t)ns * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(th.data(), mm->theta, th.size() * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(lossd);
        if (e != hipSuccess) return set_error(MXL_ERR_DEVICE, "loss read-back");
        double l = 0.0;
        for (float v : lh) l += v;
        l *= inv;
        for (int ll = 0; ll < mm->sh.nl; ++ll) {
            const int w0 = mm->sh.off[ll], w1 = w0 + mm->sh.dims[ll] * mm->sh.dims[ll + 1];
            for (int j = w0; j < w1; ++j) l += (double)lambda * th[j] * th[j];
        }
        mm->loss = (float)l;
        if (loss_host) *loss_host = mm->loss;
    }
    return MXL_OK;
}

extern "C" mxl_status mxl_mlp_forward(const mxl_mlp *mm, int64_t ns, const float *X, float *Y) try {
    if (!Y) return set_error(MXL_ERR_INVALID_ARG, "Y required");
    return mlp_run(const_cast<mxl_mlp *>(mm), ns, X, nullptr, nullptr, 0.f, Y, nullptr, false);
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_mlp_loss_grad(mxl_mlp *mm, int64_t ns, const float *X, const float *T,
                                        const float *M, float lambda, float *loss_host) try {
    if (!T || !M) return set_error(MXL_ERR_INVALID_ARG, "targets and mask required");
    return mlp_run(mm, ns, X, T, M, lambda, nullptr, loss_host, true);
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_mlp_adam_step(mxl_mlp *mm, int64_t t, float lr, float beta1, float beta2,
                                        float eps) try {
    if (!mm || t < 1) return set_error(MXL_ERR_INVALID_ARG, "network and step t >= 1");
    const float c1 = 1.f - (float)std::pow((double)beta1, (double)t);
    const float c2 = 1.f - (float)std::pow((double)beta2, (double)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((mm->sh.nparams + 255) / 256)), dim3(256), 0, mm->ctx->stream,
                       mm->sh.nparams, (float *)mm->theta, (const float *)mm->grad, (float *)mm->m,
                       (float *)mm->v, lr, beta1, beta2, eps, c1, c2);
    if (hipGetLastError() != hipSuccess) return set_error(MXL_ERR_DEVICE, "adam launch");
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_mlp_destroy(mxl_mlp *mm) try {
    if (!mm) return MXL_OK;
    if (mm->ctx) (void)hipStreamSynchronize(mm->ctx->stream);
    (void)hipFree(mm->theta);
    (void)hipFree(mm->grad);
    (void)hipFree(mm->m);
    (void)hipFree(mm->v);
    (void)hipFree(mm->gs);
    delete mm;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

// ================================================================ selector
struct mxl_selector {
    CtxRef ctx;
    std::vector<mxl_kernel_class> classes;
    mxl_mlp *net = nullptr;
    double mean[16], sd[16];
    uint32_t log_mask = 0;
    double delta = 0.05, zmax = 4.0;
    void *dz = nullptr, *ds = nullptr;  // one standardised feature row, one score row
};

extern "C" mxl_status mxl_selector_create(mxl_ctx *ctx, int32_t nclasses, const mxl_kernel_class *classes,
                                          int32_t nlayers, const int32_t *dims, const float *theta_host,
                                          const double *mean16, const double *std16, uint32_t log_mask,
                                          double delta, double zmax, mxl_selector **out) try {
    if (!ctx || !classes || !dims || !theta_host || !mean16 || !std16 || !out || nclasses < 1 ||
        nclasses > kMlpMaxW || nlayers < 1 || nlayers > kMlpMaxL)
        return set_error(MXL_ERR_INVALID_ARG, "selector: context, 1..64 classes, network and statistics required");
    *out = nullptr;
    if (dims[0] != 16 || dims[nlayers] != nclasses)
        return set_error(MXL_ERR_DIM_MISMATCH, "selector network must map 16 features to one score per class");
    for (int c = 0; c < nclasses; ++c) {
        const int f = classes[c].format;
        if (f < MXL_FMT_CSR || f > MXL_FMT_HYB) return set_error(MXL_ERR_INVALID_ARG, "selector: unknown format");
    }
    for (int j = 0; j < 16; ++j)
        if (!(std16[j] > 0.0) || !std::isfinite(mean16[j]))
            return set_error(MXL_ERR_INVALID_ARG, "selector: std must be positive, mean finite");
    DeviceScope dsc(ctx->device);
    auto *S = new mxl_selector;
    S->ctx = ctx;
    S->classes.assign(classes, classes + nclasses);
    for (int j = 0; j < 16; ++j) {
        S->mean[j] = mean16[j];
        S->sd[j] = std16[j];
    }
    S->log_mask = log_mask;
    S->delta = delta;
    S->zmax = zmax;
    mxl_status st = mxl_mlp_create(ctx, nlayers, dims, theta_host, &S->net);
    if (st != MXL_OK) {
        delete S;
        return st;
    }
    if (hipMalloc(&S->dz, 16 * 4) != hipSuccess || hipMalloc(&S->ds, (size_t)nclasses * 4) != hipSuccess) {
        mxl_selector_destroy(S);
        return set_error(MXL_ERR_OUT_OF_MEMORY, "selector buffers");
    }
    *out = S;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

extern "C" mxl_status mxl_selector_destroy(mxl_selector *S) try {
    if (!S) return MXL_OK;
    {
        DeviceScope dsc(S->ctx->device);
        mxl_mlp_destroy(S->net);
        (void)hipFree(S->dz);
        (void)hipFree(S->ds);
    }
    delete S;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

namespace {

// Width of the padded part a class needs (-1: not padded).
int64_t class_width(const mxl_kernel_class &k, const std::vector<unsigned> &hist, int64_t n) {
    if (k.format != MXL_FMT_ELL && k.format != MXL_FMT_HYB) return -1;
    if (n == 0) return 0;
    if (k.format == MXL_FMT_ELL) return (int64_t)hist.size() - 1;
    const double q = k.params.hyb_quantile > 0 ? k.params.hyb_quantile : 0.9;
    const int64_t rank = quantile_rank(std::min(q, 1.0), n);
    int64_t cum = 0;
    for (size_t L = 0; L < hist.size(); ++L) {
        cum += hist[L];
        if (cum >= rank) return (int64_t)L;
    }
    return (int64_t)hist.size() - 1;
}

}  // namespace

extern "C" mxl_status mxl_select(const mxl_selector *S, const mxl_op *Aop, int32_t mode, const void *x,
                                 void *y, int32_t reps, int32_t *class_out, double *scores,
                                 double *times_ms, mxl_select_info *info) try {
    if (!S || !Aop || Aop->kind != MXL_OP_MATRIX || !class_out)
        return set_error(MXL_ERR_INVALID_ARG, "selector, matrix operator and class output required");
    if (mode != MXL_SELECT_MODEL && mode != MXL_SELECT_EXHAUSTIVE && mode != MXL_SELECT_MODEL_FALLBACK)
        return set_error(MXL_ERR_INVALID_ARG, "unknown selection mode");
    if (mode == MXL_SELECT_EXHAUSTIVE && (!x || !y))
        return set_error(MXL_ERR_INVALID_ARG, "exhaustive selection needs x and y to time with");
    if (Aop->mat->ctx->device != S->ctx->device)
        return set_error(MXL_ERR_INVALID_ARG, "matrix and selector live on different devices");
    if (Aop->mat->format == MXL_FMT_STENCIL)
        return set_error(MXL_ERR_NOT_IMPLEMENTED, "a matrix-free stencil has no formats to choose from");
    if ((x || y) && reps < 1) return set_error(MXL_ERR_INVALID_ARG, "reps must be >= 1");
    const MatrixImpl &A = *Aop->mat;
    DeviceScope dsc(S->ctx->device);
    const int C = (int)S->classes.size();
    const double inf = std::numeric_limits<double>::infinity(), nan = std::nan("");
    mxl_select_info inf_out{};
    double f[16];
    std::vector<unsigned> hist;
    int64_t maxbw = 0;
    mxl_status st = features_compute(A, f, &hist, &maxbw);
    if (st != MXL_OK) return st;
    if (hist.empty()) hist.assign(1, (unsigned)A.nrows);
    std::vector<bool> feasible(C);
    for (int c = 0; c < C; ++c) {
        const mxl_kernel_class &k = S->classes[c];
        const int64_t w = class_width(k, hist, A.nrows);
        feasible[c] = w < 0 || ell_fits(A, w);
        if (k.format == MXL_FMT_ELL && k.params.variant == MXL_ELL_DELTA16 && maxbw > 32767) feasible[c] = false;
    }
    // standardised features and their largest magnitude
    float z[16];
    double maxz = 0.0;
    for (int j = 0; j < 16; ++j) {
        const double phi = (S->log_mask >> j) & 1u ? std::log1p(std::max(f[j], 0.0)) : f[j];
        const double zj = (phi - S->mean[j]) / S->sd[j];
        z[j] = (float)zj;
        maxz = std::max(maxz, std::fabs(zj));
    }
    inf_out.max_z = maxz;
    std::vector<double> sc(C, nan), tm(C, nan);
    std::vector<int> order;
    if (mode != MXL_SELECT_EXHAUSTIVE) {
        std::vector<float> out((size_t)C);
        hipStream_t s = S->ctx->stream;
        if (hipMemcpyAsync(S->dz, z, sizeof z, hipMemcpyHostToDevice, s) != hipSuccess)
            return set_error(MXL_ERR_DEVICE, "selector feature upload");
        if ((st = mxl_mlp_forward(S->net, 1, (const float *)S->dz, (float *)S->ds)) != MXL_OK) return st;
        if (hipMemcpyAsync(out.data(), S->ds, (size_t)C * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return set_error(MXL_ERR_DEVICE, "selector score read-back");
        for (int c = 0; c < C; ++c) sc[c] = feasible[c] ? (double)out[c] : inf;
        for (int c = 0; c < C; ++c)
            if (feasible[c]) order.push_back(c);
        // stable order by score, ties to the lower class index
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sc[a] < sc[b]; });
        if (order.empty()) return set_error(MXL_ERR_INFEASIBLE_FORMAT, "no feasible class");
        inf_out.margin = order.size() > 1 ? sc[order[1]] - sc[order[0]] : inf;
    } else {
        for (int c = 0; c < C; ++c)
            if (feasible[c]) order.push_back(c);
        if (order.empty()) return set_error(MXL_ERR_INFEASIBLE_FORMAT, "no feasible class");
        inf_out.margin = inf;
    }
    std::vector<int> timed;
    if (mode == MXL_SELECT_EXHAUSTIVE) {
        timed = order;
    } else if (mode == MXL_SELECT_MODEL_FALLBACK && x && y &&
               (inf_out.margin < S->delta || maxz > S->zmax || std::isnan(inf_out.margin))) {
        for (size_t k = 0; k < order.size() && k < 3; ++k) timed.push_back(order[k]);
    }
    int choice = order[0];
    if (!timed.empty()) {
        double best = inf;
        int nt = 0;
        for (int c : timed) {
            const mxl_kernel_class &k = S->classes[c];
            mxl_op *op = nullptr;
            st = mxl_convert(Aop, (mxl_format)k.format, &k.params, &op);
            if (st == MXL_ERR_INFEASIBLE_FORMAT) continue;
            if (st != MXL_OK) return st;
            double ms = 0.0;
            st = mxl_time_apply(op, x, y, reps, 1, &ms);
            mxl_op_destroy(op);
            if (st != MXL_OK) return st;
            tm[c] = ms;
            ++nt;
            if (ms < best) {
                best = ms;
                choice = c;
            }
        }
        if (nt == 0) return set_error(MXL_ERR_INFEASIBLE_FORMAT, "no timed class could be built");
        inf_out.fallback = 1;
        inf_out.ntimed = nt;
        inf_out.best_ms = best;
    }
    *class_out = choice;
    if (scores)
        for (int c = 0; c < C; ++c) scores[c] = sc[c];
    if (times_ms)
        for (int c = 0; c < C; ++c) times_ms[c] = tm[c];
    if (info) *info = inf_out;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}
