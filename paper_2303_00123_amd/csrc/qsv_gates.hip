// Unfused gate kernels: one HBM pass per gate (Algs. 1-3 of Sec. 2), plus
// state initialisation.  Positions p are index-bit positions (p = n-1-q for
// qubit q under Definition 1).
#include "qsv_common.h"
#include "qsv_internal.h"

namespace qsv {
namespace {

constexpr int kThreads = 256;

// Pairs per thread: enough independent 16-byte loads in flight per thread to
// cover HBM latency (4 pairs = 8 loads for c128, 8 pairs = 16 loads for c64).
template <typename R>
struct PPT;
template <>
struct PPT<double> { static constexpr int value = 4; };
template <>
struct PPT<float> { static constexpr int value = 8; };

// Gate kernels: pairs (quads) per thread.  Few per thread and many
// workgroups, with non-temporal loads and stores (the state streams through
// once per gate, so it should not displace other lines from the caches),
// measured best on MI355X: 67-77 % of the HBM peak at 30 qubits against
// 65-67 % with 4 pairs per thread and ordinary accesses.
template <typename R>
struct GatePairs;
template <>
struct GatePairs<double> { static constexpr int value = 1; };
template <>
struct GatePairs<float> { static constexpr int value = 2; };
template <typename R>
struct GateQuads { static constexpr int value = 1; };

// ---------------------------------------------------------------- |b>
template <typename R>
__global__ __launch_bounds__(kThreads) void k_init_basis(typename V2T<R>::type* __restrict__ s,
                                                         uint64_t N, uint64_t b) {
    using V = typename V2T<R>::type;
    constexpr int P = PPT<R>::value;
    constexpr uint64_t BS = uint64_t(kThreads) * P;
    for (uint64_t blk = blockIdx.x; blk * BS < N; blk += gridDim.x) {
        const uint64_t i0 = blk * BS + threadIdx.x;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint64_t i = i0 + uint64_t(k) * kThreads;
            if (i < N) {
                V v;
                v.x = (i == b) ? R(1) : R(0);
                v.y = R(0);
                s[i] = v;
            }
        }
    }
}

// ------------------------------------------------------------- Alg. 1
// Pair j -> a_j = insert0(j, p), b_j = a_j + 2^p; 2x2 matvec in place.
// CTRL: Alg. 2 with its control at a low index bit pc (below the 128-byte
// line): every pair over the target is read and written, and U applies
// where bit pc of a_j equals cs.  The pairs Alg. 2 would skip share lines
// with the ones it moves, so HBM carries the whole state either way; this
// form keeps every access a full, contiguous line.
template <typename R, bool CTRL = false>
__global__ __launch_bounds__(kThreads) void k_apply1q(typename V2T<R>::type* __restrict__ s,
                                                      uint64_t npairs, int p, M2<R> u, int pc = 0,
                                                      int cs = 0) {
    using V = typename V2T<R>::type;
    constexpr int P = GatePairs<R>::value;
    constexpr uint64_t BS = uint64_t(kThreads) * P;
    for (uint64_t blk = blockIdx.x; blk * BS < npairs; blk += gridDim.x) {
        const uint64_t j0 = blk * BS + threadIdx.x;
        const uint64_t w = uint64_t(1) << p;
        V a[P], b[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint64_t j = j0 + uint64_t(k) * kThreads;
            if (j < npairs) {
                const uint64_t ia = insert0(j, p);
                a[k] = ld_nt(s + ia);
                b[k] = ld_nt(s + ia + w);
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint64_t j = j0 + uint64_t(k) * kThreads;
            if (j < npairs) {
                const uint64_t ia = insert0(j, p);
                V oa, ob;
                mv2(u.v, a[k], b[k], oa, ob);
                if (CTRL && int((ia >> pc) & 1) != cs) {
                    oa = a[k];
                    ob = b[k];
                }
                st_nt(s + ia, oa);
                st_nt(s + ia + w, ob);
            }
        }
    }
}

// ------------------------------------------------------------- Alg. 2
// Pair j -> zero bits inserted at both positions (lower first), the control
// bit set to cs, b_j = a_j + 2^pt.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_applyc1q(typename V2T<R>::type* __restrict__ s,
                                                       uint64_t npairs, int plo, int phi, int pc,
                                                       int pt, int cs, M2<R> u) {
    using V = typename V2T<R>::type;
    constexpr int P = GatePairs<R>::value;
    constexpr uint64_t BS = uint64_t(kThreads) * P;
    for (uint64_t blk = blockIdx.x; blk * BS < npairs; blk += gridDim.x) {
        const uint64_t j0 = blk * BS + threadIdx.x;
        const uint64_t wt = uint64_t(1) << pt;
        const uint64_t wc = cs ? (uint64_t(1) << pc) : 0;
        V a[P], b[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint64_t j = j0 + uint64_t(k) * kThreads;
            if (j < npairs) {
                const uint64_t ia = insert0(insert0(j, plo), phi) | wc;
                a[k] = ld_nt(s + ia);
                b[k] = ld_nt(s + ia + wt);
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint64_t j = j0 + uint64_t(k) * kThreads;
            if (j < npairs) {
                const uint64_t ia = insert0(insert0(j, plo), phi) | wc;
                V oa, ob;
                mv2(u.v, a[k], b[k], oa, ob);
                st_nt(s + ia, oa);
                st_nt(s + ia + wt, ob);
            }
        }
    }
}

// ------------------------------------------------------------- Alg. 3
// Quad j -> base with zero bits at both positions; element r (= 2*x_qa + x_qb)
// adds the qa weight if r >> 1 and the qb weight if r & 1.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_apply2q(typename V2T<R>::type* __restrict__ s,
                                                      uint64_t nquads, int plo, int phi, int pa,
                                                      int pb, M4<R> u) {
    using V = typename V2T<R>::type;
    constexpr int P = GateQuads<R>::value;
    constexpr uint64_t BS = uint64_t(kThreads) * P;
    for (uint64_t blk = blockIdx.x; blk * BS < nquads; blk += gridDim.x) {
        const uint64_t j0 = blk * BS + threadIdx.x;
        const uint64_t wa = uint64_t(1) << pa, wb = uint64_t(1) << pb;
        V v[P][4];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint64_t j = j0 + uint64_t(k) * kThreads;
            if (j < nquads) {
                const uint64_t i0 = insert0(insert0(j, plo), phi);
                v[k][0] = ld_nt(s + i0);
                v[k][1] = ld_nt(s + i0 + wb);
                v[k][2] = ld_nt(s + i0 + wa);
                v[k][3] = ld_nt(s + i0 + wa + wb);
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint64_t j = j0 + uint64_t(k) * kThreads;
            if (j < nquads) {
                const uint64_t i0 = insert0(insert0(j, plo), phi);
                V o[4];
                mv4(u.v, v[k], o);
                st_nt(s + i0, o[0]);
                st_nt(s + i0 + wb, o[1]);
                st_nt(s + i0 + wa, o[2]);
                st_nt(s + i0 + wa + wb, o[3]);
            }
        }
    }
}

template <typename R>
unsigned grid_for(uint64_t items, int per_thread) {
    const uint64_t per_block = uint64_t(kThreads) * per_thread;
    return capped_grid((items + per_block - 1) / per_block);
}

template <typename R>
M2<R> to_m2(const double* u) {
    M2<R> m;
    for (int i = 0; i < 8; ++i) m.v[i] = R(u[i]);
    return m;
}
template <typename R>
M4<R> to_m4(const double* u) {
    M4<R> m;
    for (int i = 0; i < 32; ++i) m.v[i] = R(u[i]);
    return m;
}

template <typename R>
hipError_t init_basis_t(qsv_ctx ctx, void* s, int n, uint64_t b) {
    using V = typename V2T<R>::type;
    const uint64_t N = uint64_t(1) << n;
    prof_before(ctx, sizeof(R) == 8 ? "init_basis_c128" : "init_basis_c64", double(N) * sizeof(V));
    hipLaunchKernelGGL(k_init_basis<R>, dim3(grid_for<R>(N, PPT<R>::value)), dim3(kThreads), 0,
                       ctx->stream, static_cast<V*>(s), N, b);
    prof_after(ctx);
    return hipGetLastError();
}

template <typename R>
hipError_t apply1q_t(qsv_ctx ctx, void* s, int n, int p, const double* u) {
    using V = typename V2T<R>::type;
    const uint64_t np = uint64_t(1) << (n - 1);
    prof_before(ctx, sizeof(R) == 8 ? "apply1q_c128" : "apply1q_c64",
                2.0 * double(uint64_t(1) << n) * sizeof(V));
    hipLaunchKernelGGL((k_apply1q<R, false>), dim3(grid_for<R>(np, GatePairs<R>::value)), dim3(kThreads), 0,
                       ctx->stream, static_cast<V*>(s), np, p, to_m2<R>(u), 0, 0);
    prof_after(ctx);
    return hipGetLastError();
}

template <typename R>
hipError_t applyc1q_t(qsv_ctx ctx, void* s, int n, int pc, int pt, int cs, const double* u) {
    using V = typename V2T<R>::type;
    const uint64_t np = uint64_t(1) << (n - 2);
    const int plo = pc < pt ? pc : pt, phi = pc < pt ? pt : pc;
    prof_before(ctx, sizeof(R) == 8 ? "applyc1q_c128" : "applyc1q_c64",
                double(uint64_t(1) << n) * sizeof(V));
    // a control below the 128-byte line: the whole state moves anyway, so
    // move it in full lines (see k_apply1q)
    const int line_bits = sizeof(R) == 8 ? 3 : 4;
    if (pc < line_bits)
        hipLaunchKernelGGL((k_apply1q<R, true>), dim3(grid_for<R>(2 * np, GatePairs<R>::value)),
                           dim3(kThreads), 0, ctx->stream, static_cast<V*>(s), 2 * np, pt,
                           to_m2<R>(u), pc, cs);
    else
        hipLaunchKernelGGL(k_applyc1q<R>, dim3(grid_for<R>(np, GatePairs<R>::value)), dim3(kThreads), 0,
                           ctx->stream, static_cast<V*>(s), np, plo, phi, pc, pt, cs, to_m2<R>(u));
    prof_after(ctx);
    return hipGetLastError();
}

template <typename R>
hipError_t apply2q_t(qsv_ctx ctx, void* s, int n, int pa, int pb, const double* u) {
    using V = typename V2T<R>::type;
    const uint64_t nq = uint64_t(1) << (n - 2);
    const int plo = pa < pb ? pa : pb, phi = pa < pb ? pb : pa;
    prof_before(ctx, sizeof(R) == 8 ? "apply2q_c128" : "apply2q_c64",
                2.0 * double(uint64_t(1) << n) * sizeof(V));
    hipLaunchKernelGGL(k_apply2q<R>, dim3(grid_for<R>(nq, GateQuads<R>::value)), dim3(kThreads), 0,
                       ctx->stream, static_cast<V*>(s), nq, plo, phi, pa, pb, to_m4<R>(u));
    prof_after(ctx);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init_basis(qsv_ctx ctx, void* s, int n, int dtype, uint64_t b) {
    return dtype == QSV_C128 ? init_basis_t<double>(ctx, s, n, b) : init_basis_t<float>(ctx, s, n, b);
}
hipError_t launch_apply1q(qsv_ctx ctx, void* s, int n, int dtype, int p, const double* u) {
    return dtype == QSV_C128 ? apply1q_t<double>(ctx, s, n, p, u) : apply1q_t<float>(ctx, s, n, p, u);
}
hipError_t launch_applyc1q(qsv_ctx ctx, void* s, int n, int dtype, int pc, int pt, int cs,
                           const double* u) {
    return dtype == QSV_C128 ? applyc1q_t<double>(ctx, s, n, pc, pt, cs, u)
                             : applyc1q_t<float>(ctx, s, n, pc, pt, cs, u);
}
hipError_t launch_apply2q(qsv_ctx ctx, void* s, int n, int dtype, int pa, int pb, const double* u) {
    return dtype == QSV_C128 ? apply2q_t<double>(ctx, s, n, pa, pb, u)
                             : apply2q_t<float>(ctx, s, n, pa, pb, u);
}
hipError_t launch_gate(qsv_ctx ctx, void* s, int n, int dtype, const PGate& g) {
    switch (g.kind) {
    case QSV_G1Q: return launch_apply1q(ctx, s, n, dtype, g.p0, g.m);
    case QSV_GC1Q: return launch_applyc1q(ctx, s, n, dtype, g.p0, g.p1, g.cs, g.m);
    case QSV_G2Q: return launch_apply2q(ctx, s, n, dtype, g.p0, g.p1, g.m);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qsv
