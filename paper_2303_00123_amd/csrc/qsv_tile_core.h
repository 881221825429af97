// Device core shared by the tile-pass kernels (single-state passes and the
// batched persistent kernel): the LDS swizzle, bit deposit helpers, the
// compile-time register gate bodies (index maps of Algs. 1-3 resolved per
// register bit), their runtime dispatch, and the stage loop.
#pragma once

#include <type_traits>

#include "qsv_common.h"
#include "qsv_internal.h"

namespace qsv {
namespace tile {

constexpr int kThreads = kTileThreads;

template <typename R>
struct TileK;
template <>
struct TileK<double> { static constexpr int value = 13; };   // 8192 x 16 B = 128 KiB
template <>
struct TileK<float> { static constexpr int value = 13; };    // 8192 x 8 B = 64 KiB

template <typename R>
__device__ __forceinline__ uint32_t swz(uint32_t e) {
    return tile_swz(e, int(sizeof(typename V2T<R>::type)));
}

// Deposit the low `k` bits of e at the positions pos[0..k).
__device__ __forceinline__ uint64_t deposit(uint32_t e, const int32_t* pos, int k) {
    uint64_t off = 0;
    for (int i = 0; i < k; ++i)
        if ((e >> i) & 1u) off |= uint64_t(1) << pos[i];
    return off;
}
__device__ __forceinline__ uint32_t deposit32(uint32_t e, const int32_t* pos, int k) {
    uint32_t off = 0;
    for (int i = 0; i < k; ++i)
        if ((e >> i) & 1u) off |= 1u << pos[i];
    return off;
}

template <int B>
using IC = std::integral_constant<int, B>;

// ---------------------------------------------------- register gate bodies
template <int B, typename R, typename V, int P>
__device__ __forceinline__ void rg_1q(V (&v)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (!(i & (1 << B))) {
            const V a = v[i], b = v[i | (1 << B)];
            mv2(m, a, b, v[i], v[i | (1 << B)]);
        }
}

template <typename R, typename V>
__device__ __forceinline__ V cmul(const V& a, R dr, R di) {
    V o;
    o.x = a.x * dr - a.y * di;
    o.y = a.x * di + a.y * dr;
    return o;
}

template <int B, typename R, typename V, int P>
__device__ __forceinline__ void rg_1d(V (&v)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
        if (i & (1 << B)) v[i] = cmul(v[i], m[2], m[3]);
        else v[i] = cmul(v[i], m[0], m[1]);
    }
}

template <int C, int T, int CS, typename R, typename V, int P>
__device__ __forceinline__ void rg_c1q(V (&v)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (((i >> C) & 1) == CS && !(i & (1 << T))) {
            const V a = v[i], b = v[i | (1 << T)];
            mv2(m, a, b, v[i], v[i | (1 << T)]);
        }
}

template <int C, int T, int CS, typename V, int P>
__device__ __forceinline__ void rg_cx(V (&v)[P]) {
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (((i >> C) & 1) == CS && !(i & (1 << T))) {
            const V a = v[i];
            v[i] = v[i | (1 << T)];
            v[i | (1 << T)] = a;
        }
}

template <int C, int T, int CS, typename R, typename V, int P>
__device__ __forceinline__ void rg_cd(V (&v)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (((i >> C) & 1) == CS) {
            if (i & (1 << T)) v[i] = cmul(v[i], m[2], m[3]);
            else v[i] = cmul(v[i], m[0], m[1]);
        }
}

template <int A, int B, typename R, typename V, int P>
__device__ __forceinline__ void rg_2q(V (&v)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (!(i & (1 << A)) && !(i & (1 << B))) {
            V in[4], out[4];
            in[0] = v[i];
            in[1] = v[i | (1 << B)];
            in[2] = v[i | (1 << A)];
            in[3] = v[i | (1 << A) | (1 << B)];
            mv4(m, in, out);
            v[i] = out[0];
            v[i | (1 << B)] = out[1];
            v[i | (1 << A)] = out[2];
            v[i | (1 << A) | (1 << B)] = out[3];
        }
}

// ------------------------------------------------------ runtime dispatch
template <int RB, typename F>
__device__ __forceinline__ void on_bit(int b, F&& f) {
    switch (b) {
    case 0: f(IC<0>{}); break;
    case 1: f(IC<1>{}); break;
    case 2: if constexpr (RB > 2) f(IC<2>{}); break;
    case 3: if constexpr (RB > 3) f(IC<3>{}); break;
    case 4: if constexpr (RB > 4) f(IC<4>{}); break;
    case 5: if constexpr (RB > 5) f(IC<5>{}); break;
    default: break;
    }
}

// Controlled kinds are emitted for control state 1 only (the host lowers a
// control-state-0 gate to a 2-qubit gate), and 2-qubit gates with r0 < r1
// (the host permutes the matrix), which keeps the number of compiled
// specialisations -- and the kernel's instruction footprint -- small.
template <int RB, typename R, typename V, int P>
__device__ __forceinline__ void apply_gate(V (&v)[P], const TGate<R>& g) {
    const int kind = g.kind;
    if (kind == DK_1Q) {
        on_bit<RB>(g.r0, [&](auto B) __attribute__((always_inline)) { rg_1q<decltype(B)::value>(v, g.m); });
    } else if (kind == DK_1D) {
        on_bit<RB>(g.r0, [&](auto B) __attribute__((always_inline)) { rg_1d<decltype(B)::value>(v, g.m); });
    } else if (kind == DK_2Q) {
        on_bit<RB>(g.r0, [&](auto A) __attribute__((always_inline)) {
            on_bit<RB>(g.r1, [&](auto B) __attribute__((always_inline)) {
                if constexpr (decltype(A)::value < decltype(B)::value)
                    rg_2q<decltype(A)::value, decltype(B)::value>(v, g.m);
            });
        });
    } else {
        on_bit<RB>(g.r0, [&](auto C) __attribute__((always_inline)) {
            on_bit<RB>(g.r1, [&](auto T) __attribute__((always_inline)) {
                constexpr int c = decltype(C)::value, t = decltype(T)::value;
                if constexpr (c != t) {
                    if (kind == DK_CX) rg_cx<c, t, 1>(v);
                    else if (kind == DK_CD) rg_cd<c, t, 1>(v, g.m);
                    else rg_c1q<c, t, 1>(v, g.m);
                }
            });
        });
    }
}

template <int RB, typename R, typename V, int P>
__device__ __forceinline__ void apply_range(V (&v)[P], const TGate<R>* __restrict__ gates, int gb,
                                            int ge) {
    for (int g = gb; g < ge; ++g) apply_gate<RB>(v, gates[g]);
}

// Run stages of a pass on the register-resident amplitudes v: stage 0 and
// the last stage use the load mapping; stages in between re-map through LDS.
// Ends with every thread done reading LDS if the pass used it (the caller
// may reuse `lds` right away only after its own barrier).
template <typename R, int K, int RB, typename V>
__device__ __forceinline__ void run_stages(V (&v)[1 << RB], char* lds, const TStage* stg,
                                           int nst, const TGate<R>* gates, uint32_t tid) {
    constexpr int TB = K - RB;
    constexpr int P = 1 << RB;
    constexpr uint32_t ES = sizeof(V);
    for (int st = 0; st < nst; ++st) {
        const TStage& S = stg[st];
        // LDS byte address of slot u = swz(eb | du) * ES = swz(eb) * ES ^ su[u]
        const uint32_t sb = swz<R>(deposit32(tid, S.tbits, TB)) * ES;
        if (st > 0) {
#pragma unroll
            for (int u = 0; u < P; ++u) v[u] = *reinterpret_cast<const V*>(lds + (sb ^ S.su[u]));
        }
        apply_range<RB>(v, gates, S.gbeg, S.gend);
        if (st < nst - 1) {
#pragma unroll
            for (int u = 0; u < P; ++u) *reinterpret_cast<V*>(lds + (sb ^ S.su[u])) = v[u];
            __syncthreads();
        }
    }
}

}  // namespace tile
}  // namespace qsv
