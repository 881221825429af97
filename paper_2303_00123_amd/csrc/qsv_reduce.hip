// Reductions over the state: Z-string expectations, norm, single-qubit
// probabilities, inner products, and measurement collapse.  Accumulation is
// FP64 for both state precisions, in a fixed two-stage tree (per-block
// partials, then one block), so results are bit-reproducible for a given n.
#include <mutex>

#include "qsv_common.h"
#include "qsv_internal.h"

namespace qsv {
namespace {

constexpr int kThreads = 256;
constexpr int kTermsPerPass = 16;
constexpr int kMaxBlocks = 2048;
// loads each thread keeps in flight; the sums keep the order of the plain
// strided loop, so results do not depend on it
constexpr int kUnroll = 4;

struct ZMasks {
    uint64_t m[kTermsPerPass];
    int nt;
};

// Number of stage-1 blocks for a 2^n reduction: a power of two, fixed by n.
inline unsigned red_blocks(uint64_t N) {
    uint64_t g = N / 4096;
    if (g < 1) g = 1;
    if (g > kMaxBlocks) g = kMaxBlocks;
    return unsigned(g);
}

// Fixed-order tree over the block's threads; red holds NT x kThreads values.
template <int NT>
__device__ void block_tree(double (*red)[kThreads], double* out) {
    for (int stride = kThreads / 2; stride > 0; stride >>= 1) {
        __syncthreads();
        if (int(threadIdx.x) < stride) {
#pragma unroll
            for (int t = 0; t < NT; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + stride];
        }
    }
    __syncthreads();
    if (threadIdx.x < NT) out[threadIdx.x] = red[threadIdx.x][0];
}

template <typename R>
__device__ __forceinline__ double prob(const typename V2T<R>::type& v) {
    const double x = double(v.x), y = double(v.y);
    return x * x + y * y;
}

// out[t] over this block's contiguous chunk: sum |s_x|^2 (-1)^{popc(x & m_t)}
template <typename R>
__global__ __launch_bounds__(kThreads) void k_zstr(const typename V2T<R>::type* __restrict__ s,
                                                   uint64_t N, uint64_t chunk, ZMasks zm,
                                                   double* __restrict__ partials) {
    __shared__ double red[kTermsPerPass][kThreads];
    double acc[kTermsPerPass];
#pragma unroll
    for (int t = 0; t < kTermsPerPass; ++t) acc[t] = 0.0;
    const uint64_t lo = uint64_t(blockIdx.x) * chunk;
    const uint64_t hi = lo + chunk < N ? lo + chunk : N;
    auto add = [&](uint64_t x, const typename V2T<R>::type& v) {
        const double p = prob<R>(v);
#pragma unroll
        for (int t = 0; t < kTermsPerPass; ++t)
            if (t < zm.nt) acc[t] += (__popcll(x & zm.m[t]) & 1) ? -p : p;
    };
    uint64_t x = lo + threadIdx.x;
    for (; x + (kUnroll - 1) * kThreads < hi; x += kUnroll * kThreads) {
        typename V2T<R>::type v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = s[x + u * kThreads];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) add(x + u * kThreads, v[u]);
    }
    for (; x < hi; x += kThreads) add(x, s[x]);
#pragma unroll
    for (int t = 0; t < kTermsPerPass; ++t) red[t][threadIdx.x] = acc[t];
    block_tree<kTermsPerPass>(red, partials + size_t(blockIdx.x) * kTermsPerPass);
}

// out[0] = sum over bit p clear, out[1] = bit p set
template <typename R>
__global__ __launch_bounds__(kThreads) void k_split(const typename V2T<R>::type* __restrict__ s,
                                                    uint64_t N, uint64_t chunk, int p,
                                                    double* __restrict__ partials) {
    __shared__ double red[2][kThreads];
    double a0 = 0.0, a1 = 0.0;
    const uint64_t lo = uint64_t(blockIdx.x) * chunk;
    const uint64_t hi = lo + chunk < N ? lo + chunk : N;
    auto add = [&](uint64_t x, const typename V2T<R>::type& v) {
        const double q = prob<R>(v);
        if ((x >> p) & 1) a1 += q;
        else a0 += q;
    };
    uint64_t x = lo + threadIdx.x;
    for (; x + (kUnroll - 1) * kThreads < hi; x += kUnroll * kThreads) {
        typename V2T<R>::type v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = s[x + u * kThreads];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) add(x + u * kThreads, v[u]);
    }
    for (; x < hi; x += kThreads) add(x, s[x]);
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    block_tree<2>(red, partials + size_t(blockIdx.x) * 2);
}

// <a|b> = sum conj(a_x) b_x
template <typename Ra, typename Rb>
__global__ __launch_bounds__(kThreads) void k_inner(const typename V2T<Ra>::type* __restrict__ a,
                                                    const typename V2T<Rb>::type* __restrict__ b,
                                                    uint64_t N, uint64_t chunk,
                                                    double* __restrict__ partials) {
    __shared__ double red[2][kThreads];
    double re = 0.0, im = 0.0;
    const uint64_t lo = uint64_t(blockIdx.x) * chunk;
    const uint64_t hi = lo + chunk < N ? lo + chunk : N;
    auto add = [&](const typename V2T<Ra>::type& av, const typename V2T<Rb>::type& bv) {
        const double ar = av.x, ai = av.y, br = bv.x, bi = bv.y;
        re += ar * br + ai * bi;
        im += ar * bi - ai * br;
    };
    uint64_t x = lo + threadIdx.x;
    for (; x + (kUnroll - 1) * kThreads < hi; x += kUnroll * kThreads) {
        typename V2T<Ra>::type va[kUnroll];
        typename V2T<Rb>::type vb[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            va[u] = a[x + u * kThreads];
            vb[u] = b[x + u * kThreads];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) add(va[u], vb[u]);
    }
    for (; x < hi; x += kThreads) add(a[x], b[x]);
    red[0][threadIdx.x] = re;
    red[1][threadIdx.x] = im;
    block_tree<2>(red, partials + size_t(blockIdx.x) * 2);
}

// Stage 2: out[t] = sum over blocks g of partials[g*nt_stride + t], fixed order.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_final(const double* __restrict__ partials,
                                                    int nblocks, int stride,
                                                    double* __restrict__ out) {
    __shared__ double red[NT][kThreads];
    double acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = 0.0;
    for (int g = threadIdx.x; g < nblocks; g += kThreads) {
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] += partials[size_t(g) * stride + t];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) red[t][threadIdx.x] = acc[t];
    block_tree<NT>(red, out);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_collapse(typename V2T<R>::type* __restrict__ s,
                                                       uint64_t N, int p, int keep, R scale) {
    using V = typename V2T<R>::type;
    for (uint64_t x = uint64_t(blockIdx.x) * kThreads + threadIdx.x; x < N;
         x += uint64_t(gridDim.x) * kThreads) {
        V v = s[x];
        if (int((x >> p) & 1) == keep) {
            v.x *= scale;
            v.y *= scale;
        } else {
            v.x = R(0);
            v.y = R(0);
        }
        s[x] = v;
    }
}

// Copy nt stage-2 results to the pinned host buffer and wait.
hipError_t fetch(qsv_ctx ctx, const double* dev, int nt, double* out) {
    hipError_t e = hipMemcpyAsync(ctx->h_red, dev, sizeof(double) * nt, hipMemcpyDeviceToHost,
                                  ctx->stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return e;
    for (int t = 0; t < nt; ++t) out[t] = ctx->h_red[t];
    return hipSuccess;
}

template <typename R>
hipError_t zstrings_t(qsv_ctx ctx, const void* s, int n, int nt, const uint64_t* pmasks,
                      double* out) {
    using V = typename V2T<R>::type;
    const uint64_t N = uint64_t(1) << n;
    const unsigned G = red_blocks(N);
    const uint64_t chunk = (N + G - 1) / G;
    double* partials = ctx->d_red;
    double* res = ctx->d_red + kMaxBlocks * kTermsPerPass;
    for (int t0 = 0; t0 < nt; t0 += kTermsPerPass) {
        ZMasks zm{};
        zm.nt = nt - t0 < kTermsPerPass ? nt - t0 : kTermsPerPass;
        for (int t = 0; t < zm.nt; ++t) zm.m[t] = pmasks[t0 + t];
        prof_before(ctx, sizeof(R) == 8 ? "reduce_zstr_c128" : "reduce_zstr_c64",
                    double(N) * sizeof(V));
        hipLaunchKernelGGL(k_zstr<R>, dim3(G), dim3(kThreads), 0, ctx->stream,
                           static_cast<const V*>(s), N, chunk, zm, partials);
        prof_after(ctx);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_final<kTermsPerPass>, dim3(1), dim3(kThreads), 0, ctx->stream,
                           partials, int(G), kTermsPerPass, res);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = fetch(ctx, res, zm.nt, out + t0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename R>
hipError_t split_t(qsv_ctx ctx, const void* s, int n, int p, double* out) {
    using V = typename V2T<R>::type;
    const uint64_t N = uint64_t(1) << n;
    const unsigned G = red_blocks(N);
    const uint64_t chunk = (N + G - 1) / G;
    double* partials = ctx->d_red;
    double* res = ctx->d_red + kMaxBlocks * kTermsPerPass;
    hipLaunchKernelGGL(k_split<R>, dim3(G), dim3(kThreads), 0, ctx->stream,
                       static_cast<const V*>(s), N, chunk, p, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_final<2>, dim3(1), dim3(kThreads), 0, ctx->stream, partials, int(G), 2,
                       res);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return fetch(ctx, res, 2, out);
}

template <typename Ra, typename Rb>
hipError_t inner_t(qsv_ctx ctx, const void* a, const void* b, int n, double* out) {
    using Va = typename V2T<Ra>::type;
    using Vb = typename V2T<Rb>::type;
    const uint64_t N = uint64_t(1) << n;
    const unsigned G = red_blocks(N);
    const uint64_t chunk = (N + G - 1) / G;
    double* partials = ctx->d_red;
    double* res = ctx->d_red + kMaxBlocks * kTermsPerPass;
    hipLaunchKernelGGL((k_inner<Ra, Rb>), dim3(G), dim3(kThreads), 0, ctx->stream,
                       static_cast<const Va*>(a), static_cast<const Vb*>(b), N, chunk, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_final<2>, dim3(1), dim3(kThreads), 0, ctx->stream, partials, int(G), 2,
                       res);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return fetch(ctx, res, 2, out);
}

template <typename R>
hipError_t collapse_t(qsv_ctx ctx, void* s, int n, int p, int keep, double scale) {
    using V = typename V2T<R>::type;
    const uint64_t N = uint64_t(1) << n;
    const unsigned G = capped_grid((N + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_collapse<R>, dim3(G), dim3(kThreads), 0, ctx->stream, static_cast<V*>(s),
                       N, p, keep, R(scale));
    return hipGetLastError();
}

// Copy the first nt stage-2 results to the caller's array.
__global__ void k_copy_terms(const double* __restrict__ res, int nt, double* __restrict__ out) {
    if (int(threadIdx.x) < nt) out[threadIdx.x] = res[threadIdx.x];
}

}  // namespace

// ------------------------------------------- allocation-free Z strings
// The allocation-free entry point keeps its stage-1 partials (at most 2048
// blocks x 16 terms) and the 16 stage-2 results of a pass in this fixed
// array instead of context memory: 256 KiB + 128 B of FP64.  Each GPU holds
// its own copy until the process ends.  Host code never uses the array's
// name as an address (it is a host-side stand-in): each device's address is
// looked up once with hipGetSymbolAddress and kept in g_scratch_dev.
constexpr size_t kScratchDoubles = size_t(kMaxBlocks) * kTermsPerPass + kTermsPerPass;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

void* scratch_dev(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}

template <typename R>
hipError_t zstrings_dev_t(qsv_ctx ctx, const void* s, int n, int nt, const uint64_t* qmasks,
                          double* out_dev, double* sp) {
    using V = typename V2T<R>::type;
    const uint64_t N = uint64_t(1) << n;
    const unsigned G = red_blocks(N);
    if (size_t(G) * kTermsPerPass + kTermsPerPass > kScratchDoubles) return hipErrorInvalidValue;
    const uint64_t chunk = (N + G - 1) / G;
    double* partials = sp;
    double* res = sp + size_t(kMaxBlocks) * kTermsPerPass;
    for (int t0 = 0; t0 < nt; t0 += kTermsPerPass) {
        ZMasks zm{};
        zm.nt = nt - t0 < kTermsPerPass ? nt - t0 : kTermsPerPass;
        // qubit q -> index bit n-1-q (Definition 1)
        for (int t = 0; t < zm.nt; ++t)
            for (int q = 0; q < n; ++q)
                if ((qmasks[t0 + t] >> q) & 1) zm.m[t] |= uint64_t(1) << (n - 1 - q);
        hipLaunchKernelGGL(k_zstr<R>, dim3(G), dim3(kThreads), 0, ctx->stream,
                           static_cast<const V*>(s), N, chunk, zm, partials);
        hipLaunchKernelGGL(k_final<kTermsPerPass>, dim3(1), dim3(kThreads), 0, ctx->stream,
                           partials, int(G), kTermsPerPass, res);
        hipLaunchKernelGGL(k_copy_terms, dim3(1), dim3(64), 0, ctx->stream, res, zm.nt, out_dev + t0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

hipError_t reduce_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = p;
    return hipSuccess;
}

hipError_t reduce_zstrings_dev(qsv_ctx ctx, const void* s, int n, int dtype, int nt,
                               const uint64_t* qmasks, double* out_dev) {
    double* sp = static_cast<double*>(scratch_dev(ctx->device));
    if (!sp) return hipErrorNotInitialized;
    return dtype == QSV_C128 ? zstrings_dev_t<double>(ctx, s, n, nt, qmasks, out_dev, sp)
                             : zstrings_dev_t<float>(ctx, s, n, nt, qmasks, out_dev, sp);
}

hipError_t reduce_zstrings(qsv_ctx ctx, const void* s, int n, int dtype, int nt,
                           const uint64_t* pmasks, double* out) {
    return dtype == QSV_C128 ? zstrings_t<double>(ctx, s, n, nt, pmasks, out)
                             : zstrings_t<float>(ctx, s, n, nt, pmasks, out);
}
hipError_t reduce_bit_split(qsv_ctx ctx, const void* s, int n, int dtype, int p, double* out) {
    return dtype == QSV_C128 ? split_t<double>(ctx, s, n, p, out) : split_t<float>(ctx, s, n, p, out);
}
hipError_t reduce_inner(qsv_ctx ctx, const void* a, int dta, const void* b, int dtb, int n,
                        double* out) {
    if (dta == QSV_C128 && dtb == QSV_C128) return inner_t<double, double>(ctx, a, b, n, out);
    if (dta == QSV_C128) return inner_t<double, float>(ctx, a, b, n, out);
    if (dtb == QSV_C128) return inner_t<float, double>(ctx, a, b, n, out);
    return inner_t<float, float>(ctx, a, b, n, out);
}
hipError_t launch_collapse(qsv_ctx ctx, void* s, int n, int dtype, int p, int keep, double scale) {
    return dtype == QSV_C128 ? collapse_t<double>(ctx, s, n, p, keep, scale)
                             : collapse_t<float>(ctx, s, n, p, keep, scale);
}

}  // namespace qsv
