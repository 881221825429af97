// Adjoint-method gradient sweep (Jones & Gacon, arXiv:2009.02823) over the
// gate engine: lambda = O psi, then for k = last..first
//   rotation exp(-i theta P/2):  g_k = Im <lambda| P |psi>
//   psi <- U_k^dag psi,  lambda <- U_k^dag lambda.
// Each rotation's partial sum is fused into the pass that rewinds it, so a
// rotation costs one read and one write of both vectors; per-block partials
// are reduced in a fixed order on the device, and all gradients come back
// to the host in one copy at the end.
#include <cstring>

#include "qsv_common.h"
#include "qsv_internal.h"

namespace qsv {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;

inline unsigned adj_blocks(uint64_t npairs) {
    uint64_t g = npairs / 2048;
    if (g < 1) g = 1;
    if (g > kMaxBlocks) g = kMaxBlocks;
    return unsigned(g);
}

// lambda_x = psi_x * sum_t w_t (-1)^{popc(x & m_t)}
template <typename R>
__global__ __launch_bounds__(kThreads) void k_apply_obs(const typename V2T<R>::type* __restrict__ psi,
                                                        typename V2T<R>::type* __restrict__ lam,
                                                        uint64_t N, int nt,
                                                        const uint64_t* __restrict__ masks,
                                                        const double* __restrict__ w) {
    using V = typename V2T<R>::type;
    const uint64_t x = uint64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (x >= N) return;
    double d = 0.0;
    for (int t = 0; t < nt; ++t) d += (__popcll(x & masks[t]) & 1) ? -w[t] : w[t];
    const V v = psi[x];
    V o;
    o.x = R(d * double(v.x));
    o.y = R(d * double(v.y));
    lam[x] = o;
}

// One rotation about `axis` on position p: partial Im<lam|P|psi> over this
// block's pairs, then both vectors rewound by U^dag (ud).
template <typename R, int AXIS>
__global__ __launch_bounds__(kThreads) void k_adj_rot(typename V2T<R>::type* __restrict__ psi,
                                                      typename V2T<R>::type* __restrict__ lam,
                                                      uint64_t npairs, uint64_t chunk, int p,
                                                      M2<R> ud, double* __restrict__ partials) {
    using V = typename V2T<R>::type;
    __shared__ double red[1][kThreads];
    const uint64_t w = uint64_t(1) << p;
    const uint64_t lo = uint64_t(blockIdx.x) * chunk;
    const uint64_t hi = lo + chunk < npairs ? lo + chunk : npairs;
    double acc = 0.0;
    for (uint64_t j = lo + threadIdx.x; j < hi; j += kThreads) {
        const uint64_t ia = insert0(j, p), ib = ia + w;
        const V pa = psi[ia], pb = psi[ib], la = lam[ia], lb = lam[ib];
        // (P psi)_a, (P psi)_b
        double qar, qai, qbr, qbi;
        if (AXIS == QSV_AXIS_X) {
            qar = pb.x; qai = pb.y; qbr = pa.x; qbi = pa.y;
        } else if (AXIS == QSV_AXIS_Y) {   // (-i psi_b, i psi_a)
            qar = pb.y; qai = -double(pb.x); qbr = -double(pa.y); qbi = pa.x;
        } else {                           // (psi_a, -psi_b)
            qar = pa.x; qai = pa.y; qbr = -double(pb.x); qbi = -double(pb.y);
        }
        // Im(conj(l) q) = l.x q.y - l.y q.x
        acc += double(la.x) * qai - double(la.y) * qar + double(lb.x) * qbi - double(lb.y) * qbr;
        V oa, ob;
        mv2(ud.v, pa, pb, oa, ob);
        psi[ia] = oa;
        psi[ib] = ob;
        mv2(ud.v, la, lb, oa, ob);
        lam[ia] = oa;
        lam[ib] = ob;
    }
    red[0][threadIdx.x] = acc;
    block_tree256<1>(red, partials + blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_sum_to(const double* __restrict__ partials,
                                                     int nblocks, double* __restrict__ out) {
    __shared__ double red[1][kThreads];
    double acc = 0.0;
    for (int g = threadIdx.x; g < nblocks; g += kThreads) acc += partials[g];
    red[0][threadIdx.x] = acc;
    block_tree256<1>(red, out);
}

void dagger(const PGate& g, PGate& d) {
    d = g;
    const int n = g.kind == QSV_G2Q ? 4 : 2;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            d.m[2 * (r * n + c)] = g.m[2 * (c * n + r)];
            d.m[2 * (r * n + c) + 1] = -g.m[2 * (c * n + r) + 1];
        }
}

template <typename R>
hipError_t adjoint_t(qsv_ctx ctx, void* psi, void* lam, int n, const std::vector<PGate>& fwd,
                     const std::vector<int>& rot_param, const std::vector<int>& rot_axis,
                     int nterms, const uint64_t* pmasks, const double* w, double* grad_by_gate) {
    using V = typename V2T<R>::type;
    const int dt = sizeof(R) == 8 ? QSV_C128 : QSV_C64;
    const uint64_t N = uint64_t(1) << n;
    const size_t ng = fwd.size();

    // observable upload: masks then weights
    const size_t obytes = size_t(nterms) * (sizeof(uint64_t) + sizeof(double));
    void* host = nullptr;
    hipError_t e = plan_staging(ctx, obytes, &host);
    if (e != hipSuccess) return e;
    std::memcpy(host, pmasks, size_t(nterms) * sizeof(uint64_t));
    std::memcpy(static_cast<char*>(host) + size_t(nterms) * sizeof(uint64_t), w,
                size_t(nterms) * sizeof(double));
    void* dev = nullptr;
    e = plan_upload(ctx, obytes, &dev);
    if (e != hipSuccess) return e;
    const uint64_t* dmask = static_cast<const uint64_t*>(dev);
    const double* dw = reinterpret_cast<const double*>(static_cast<char*>(dev) +
                                                       size_t(nterms) * sizeof(uint64_t));
    e = ensure_aux(ctx, ng + 1);
    if (e != hipSuccess) return e;
    double* dgrad = ctx->d_aux;

    prof_before(ctx, sizeof(R) == 8 ? "adj_obs_c128" : "adj_obs_c64", 2.0 * double(N) * sizeof(V));
    hipLaunchKernelGGL(k_apply_obs<R>, dim3(unsigned((N + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, ctx->stream, static_cast<const V*>(psi), static_cast<V*>(lam), N, nterms,
                       dmask, dw);
    prof_after(ctx);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    const uint64_t npairs = N / 2;
    const unsigned G = adj_blocks(npairs);
    const uint64_t chunk = (npairs + G - 1) / G;
    bool any_rot = false;
    for (size_t kk = ng; kk-- > 0;) {
        const PGate& g = fwd[kk];
        PGate d;
        dagger(g, d);
        if (rot_param[kk] >= 0) {
            any_rot = true;
            M2<R> ud;
            for (int i = 0; i < 8; ++i) ud.v[i] = R(d.m[i]);
            prof_before(ctx, sizeof(R) == 8 ? "adj_rot_c128" : "adj_rot_c64",
                        4.0 * double(N) * sizeof(V));
            switch (rot_axis[kk]) {
            case QSV_AXIS_X:
                hipLaunchKernelGGL((k_adj_rot<R, QSV_AXIS_X>), dim3(G), dim3(kThreads), 0,
                                   ctx->stream, static_cast<V*>(psi), static_cast<V*>(lam), npairs,
                                   chunk, g.p0, ud, ctx->d_red);
                break;
            case QSV_AXIS_Y:
                hipLaunchKernelGGL((k_adj_rot<R, QSV_AXIS_Y>), dim3(G), dim3(kThreads), 0,
                                   ctx->stream, static_cast<V*>(psi), static_cast<V*>(lam), npairs,
                                   chunk, g.p0, ud, ctx->d_red);
                break;
            default:
                hipLaunchKernelGGL((k_adj_rot<R, QSV_AXIS_Z>), dim3(G), dim3(kThreads), 0,
                                   ctx->stream, static_cast<V*>(psi), static_cast<V*>(lam), npairs,
                                   chunk, g.p0, ud, ctx->d_red);
                break;
            }
            prof_after(ctx);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(kThreads), 0, ctx->stream, ctx->d_red,
                               int(G), dgrad + kk);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        } else {
            if ((e = launch_gate(ctx, psi, n, dt, d)) != hipSuccess) return e;
            if ((e = launch_gate(ctx, lam, n, dt, d)) != hipSuccess) return e;
        }
    }
    for (size_t kk = 0; kk < ng; ++kk) grad_by_gate[kk] = 0.0;
    if (any_rot) {
        std::vector<double> tmp(ng, 0.0);
        e = hipMemcpyAsync(tmp.data(), dgrad, ng * sizeof(double), hipMemcpyDeviceToHost,
                           ctx->stream);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return e;
        for (size_t kk = 0; kk < ng; ++kk)
            if (rot_param[kk] >= 0) grad_by_gate[kk] = tmp[kk];
    } else {
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t run_adjoint(qsv_ctx ctx, void* psi, void* lam, int n, int dtype,
                       const std::vector<PGate>& fwd, const std::vector<int>& rot_param,
                       const std::vector<int>& rot_axis, int nterms, const uint64_t* pmasks,
                       const double* w, double* grad_by_gate) {
    return dtype == QSV_C128
               ? adjoint_t<double>(ctx, psi, lam, n, fwd, rot_param, rot_axis, nterms, pmasks, w,
                                   grad_by_gate)
               : adjoint_t<float>(ctx, psi, lam, n, fwd, rot_param, rot_axis, nterms, pmasks, w,
                                  grad_by_gate);
}

}  // namespace qsv
