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

// Workgroup barrier that orders LDS accesses only: it waits for this
// thread's outstanding LDS operations but not for global loads, so loads
// issued ahead (the next tile's amplitudes) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------- register gate bodies
// Each body reads the amplitudes from s and writes every slot of d (slots
// the gate leaves alone are copied), so results never overwrite inputs that
// are still live and need no register copies afterwards.  Every body reads
// the amplitudes of a pair or quad before it writes them, so s and d may
// also be the same array (in-place update); the CNOT body needs to know
// which, because its two forms differ (a renaming, or a swap in place).
template <int B, typename R, typename V, int P>
__device__ __forceinline__ void rg_1q(const V (&s)[P], V (&d)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (!(i & (1 << B))) mv2(m, s[i], s[i | (1 << B)], d[i], d[i | (1 << B)]);
}

// Real 2x2 (rotations about Y, Hadamard): four real multiply-adds per pair
// component instead of eight complex ones.
template <int B, typename R, typename V, int P>
__device__ __forceinline__ void rg_1r(const V (&s)[P], V (&d)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (!(i & (1 << B))) {
            const V a = s[i], b = s[i | (1 << B)];
            V x, y;
            x.x = fmaR(m[2], b.x, m[0] * a.x);
            x.y = fmaR(m[2], b.y, m[0] * a.y);
            y.x = fmaR(m[6], b.x, m[4] * a.x);
            y.y = fmaR(m[6], b.y, m[4] * a.y);
            d[i] = x;
            d[i | (1 << B)] = y;
        }
}

// [[a, i c], [i e, g]] with a, c, e, g real (rotations about X).
template <int B, typename R, typename V, int P>
__device__ __forceinline__ void rg_1x(const V (&s)[P], V (&d)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (!(i & (1 << B))) {
            const V a = s[i], b = s[i | (1 << B)];
            V x, y;
            x.x = fmaR(-m[3], b.y, m[0] * a.x);
            x.y = fmaR(m[3], b.x, m[0] * a.y);
            y.x = fmaR(-m[5], a.y, m[6] * b.x);
            y.y = fmaR(m[5], a.x, m[6] * b.y);
            d[i] = x;
            d[i | (1 << B)] = y;
        }
}

template <typename R, typename V>
__device__ __forceinline__ V cmul(const V& a, R dr, R di) {
    V o;
    o.x = fmaR(-a.y, di, a.x * dr);
    o.y = fmaR(a.y, dr, a.x * di);
    return o;
}

template <int B, typename R, typename V, int P>
__device__ __forceinline__ void rg_1d(const V (&s)[P], V (&d)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i) d[i] = (i & (1 << B)) ? cmul(s[i], m[2], m[3]) : cmul(s[i], m[0], m[1]);
}

template <int C, int T, typename R, typename V, int P>
__device__ __forceinline__ void rg_c1q(const V (&s)[P], V (&d)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
        if (!((i >> C) & 1)) d[i] = s[i];
        else if (!(i & (1 << T))) mv2(m, s[i], s[i | (1 << T)], d[i], d[i | (1 << T)]);
    }
}

template <int C, int T, bool INPL, typename V, int P>
__device__ __forceinline__ void rg_cx(const V (&s)[P], V (&d)[P]) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
        if constexpr (!INPL) {
            d[i] = ((i >> C) & 1) ? s[i ^ (1 << T)] : s[i];
        } else if (((i >> C) & 1) && !(i & (1 << T))) {   // s is d: swap the pair
            const V a = s[i], b = s[i | (1 << T)];
            d[i] = b;
            d[i | (1 << T)] = a;
        }
    }
}

template <int C, int T, typename R, typename V, int P>
__device__ __forceinline__ void rg_cd(const V (&s)[P], V (&d)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
        if (!((i >> C) & 1)) d[i] = s[i];
        else d[i] = (i & (1 << T)) ? cmul(s[i], m[2], m[3]) : cmul(s[i], m[0], m[1]);
    }
}

template <int A, int B, typename R, typename V, int P>
__device__ __forceinline__ void rg_2q(const V (&s)[P], V (&d)[P], const R* m) {
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (!(i & (1 << A)) && !(i & (1 << B))) {
            V in[4], out[4];
            in[0] = s[i];
            in[1] = s[i | (1 << B)];
            in[2] = s[i | (1 << A)];
            in[3] = s[i | (1 << A) | (1 << B)];
            mv4(m, in, out);
            d[i] = out[0];
            d[i | (1 << B)] = out[1];
            d[i | (1 << A)] = out[2];
            d[i | (1 << A) | (1 << B)] = out[3];
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

// d = gate(s).  One flat switch over (kind, r0, r1): every reachable case
// applies a gate, so each case can produce its results directly in the
// registers the join expects.  Controlled kinds are emitted for control
// state 1 only (the host lowers a control-state-0 gate to a 2-qubit gate),
// and 2-qubit gates with r0 < r1 (the host permutes the matrix), which keeps
// the number of compiled cases -- and the instruction footprint -- small.
// `each` hands the case body every (source, destination) register-array pair
// it applies to: one state, or a state and its co-state in the same dispatch.
#define QSV_EACH(...) each([&](const auto& s, auto& d) __attribute__((always_inline)) { __VA_ARGS__; })
#define QSV_C1(KD, B)                                                          \
    case (KD) * 64 + (B) * 8:                                                  \
        if constexpr ((B) < RB) {                                              \
            if constexpr ((KD) == DK_1Q) QSV_EACH(rg_1q<(B)>(s, d, m));        \
            else if constexpr ((KD) == DK_1R) QSV_EACH(rg_1r<(B)>(s, d, m));   \
            else QSV_EACH(rg_1d<(B)>(s, d, m));                                \
        } else {                                                               \
            __builtin_unreachable();                                           \
        }                                                                      \
        break;
#define QSV_C2(KD, A, B)                                                       \
    case (KD) * 64 + (A) * 8 + (B):                                            \
        if constexpr ((A) < RB && (B) < RB && (A) != (B) && ((KD) != DK_2Q || (A) < (B))) { \
            if constexpr ((KD) == DK_2Q) QSV_EACH(rg_2q<(A), (B)>(s, d, m));   \
            else if constexpr ((KD) == DK_CX) QSV_EACH(rg_cx<(A), (B), INPL>(s, d)); \
            else if constexpr ((KD) == DK_CD) QSV_EACH(rg_cd<(A), (B)>(s, d, m)); \
            else QSV_EACH(rg_c1q<(A), (B)>(s, d, m));                          \
        } else {                                                               \
            __builtin_unreachable();                                           \
        }                                                                      \
        break;
#define QSV_C2ROW(KD, A) \
    QSV_C2(KD, A, 0) QSV_C2(KD, A, 1) QSV_C2(KD, A, 2) QSV_C2(KD, A, 3) QSV_C2(KD, A, 4) QSV_C2(KD, A, 5)
#define QSV_C2ALL(KD) \
    QSV_C2ROW(KD, 0) QSV_C2ROW(KD, 1) QSV_C2ROW(KD, 2) QSV_C2ROW(KD, 3) QSV_C2ROW(KD, 4) QSV_C2ROW(KD, 5)
#define QSV_C1ALL(KD) QSV_C1(KD, 0) QSV_C1(KD, 1) QSV_C1(KD, 2) QSV_C1(KD, 3) QSV_C1(KD, 4) QSV_C1(KD, 5)

// Opcode of a gate: kind * 64 + r0 * 8 + r1; kOpCopy is d = s.
constexpr int kOpCopy = 7 * 64;

template <typename V, int P>
__device__ __forceinline__ void copy_regs(const V (&s)[P], V (&d)[P]) {
#pragma unroll
    for (int u = 0; u < P; ++u) d[u] = s[u];
}

template <int RB, bool INPL, typename R, typename EACH>
__device__ __forceinline__ void apply_op_each(int op, const R* m, EACH&& each) {
    switch (op) {
    case kOpCopy:
        QSV_EACH(copy_regs(s, d));
        break;
        QSV_C1ALL(DK_1Q)
        QSV_C1ALL(DK_1D)
        QSV_C1ALL(DK_1R)
        QSV_C2ALL(DK_C1Q)
        QSV_C2ALL(DK_CX)
        QSV_C2ALL(DK_CD)
        QSV_C2ALL(DK_2Q)
    default: __builtin_unreachable();
    }
}

template <int RB, typename R, typename V, int P>
__device__ __forceinline__ void apply_op(const V (&s)[P], V (&d)[P], int op, const R* m) {
    apply_op_each<RB, false>(op, m, [&](auto&& f) __attribute__((always_inline)) { f(s, d); });
}

// The same gate on two states (the adjoint sweep's state and co-state),
// each updated in place.
template <int RB, typename R, typename V, int P>
__device__ __forceinline__ void apply_op2_inplace(V (&v1)[P], V (&v2)[P], int op, const R* m) {
    apply_op_each<RB, true>(op, m, [&](auto&& f) __attribute__((always_inline)) {
        f(v1, v1);
        f(v2, v2);
    });
}

#undef QSV_EACH
#undef QSV_C1ALL
#undef QSV_C2ALL
#undef QSV_C2ROW
#undef QSV_C2
#undef QSV_C1

// Gates [gb, ge) on v, two per iteration: the first writes w, the second
// writes v back, so every result lands in the registers its reader expects
// without copies; an odd count ends with a copy in place of the second.
template <int RB, typename R, typename V, int P>
__device__ __forceinline__ void apply_range(V (&v)[P], const TGate<R>* __restrict__ gates, int gb,
                                            int ge) {
    V w[P];
    for (int g = gb; g < ge; g += 2) {
        const TGate<R>& a = gates[g];
        apply_op<RB>(v, w, a.kind * 64 + a.r0 * 8 + a.r1, a.m);
        const bool two = g + 1 < ge;
        const TGate<R>& b = gates[two ? g + 1 : g];
        apply_op<RB>(w, v, two ? b.kind * 64 + b.r0 * 8 + b.r1 : kOpCopy, b.m);
    }
}

// Write the register slots u whose register bit J equals RHO to LDS.
template <int RB, int RHO, typename V>
__device__ __forceinline__ void write_half(const V (&v)[1 << RB], char* lds, uint32_t sb,
                                           const uint32_t* su, int jw) {
    on_bit<RB>(jw, [&](auto J) __attribute__((always_inline)) {
        constexpr int j = decltype(J)::value;
#pragma unroll
        for (int u = 0; u < (1 << RB); ++u)
            if (((u >> j) & 1) == RHO) *reinterpret_cast<V*>(lds + (sb ^ su[u])) = v[u];
    });
}

// Run stages of a pass on the register-resident amplitudes v: stage 0 and
// the last stage use the load and store mappings; stages in between re-map
// through LDS.  Full exchange (SPLIT false): the whole tile is written, then
// read back in the next stage's mapping.  Split exchange: consecutive stages
// share a register bit h (the next stage's last register bit), and the tile
// moves in two rounds through half of it in LDS -- the amplitudes with h = 0,
// then those with h = 1 -- so a workgroup needs half the LDS.
// Ends with every thread done reading LDS if the pass used it (the caller
// may reuse `lds` right away only after its own barrier).
template <typename R, int K, int RB, bool SPLIT = false, typename V>
__device__ __forceinline__ void run_stages(V (&v)[1 << RB], char* lds, const TStage* stg,
                                           int nst, const TGate<R>* gates, uint32_t tid) {
    constexpr int TB = K - RB;
    constexpr int P = 1 << RB;
    constexpr uint32_t ES = sizeof(V);
    if constexpr (!SPLIT) {
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
                for (int u = 0; u < P; ++u) *reinterpret_cast<V*>(lds + (sb ^ S.su_wr[u])) = v[u];
                lds_barrier();
            }
        }
    } else {
        for (int st = 0; st < nst; ++st) {
            const TStage& S = stg[st];
            apply_range<RB>(v, gates, S.gbeg, S.gend);
            if (st + 1 < nst) {
                const TStage& N = stg[st + 1];
                const uint32_t sbw = swz<R>(deposit32(tid, S.tbw, TB)) * ES;
                const uint32_t sbr = swz<R>(deposit32(tid, N.tbr, TB)) * ES;
                V w[P / 2];
                __builtin_amdgcn_s_setprio(2);   // LDS phase (see the tile kernel)
                if (st > 0) lds_barrier();   // the previous change's reads are done
                write_half<RB, 0>(v, lds, sbw, S.su_wr, S.jw);
                lds_barrier();
#pragma unroll
                for (int u = 0; u < P / 2; ++u) w[u] = *reinterpret_cast<const V*>(lds + (sbr ^ N.su[u]));
                lds_barrier();
                write_half<RB, 1>(v, lds, sbw, S.su_wr, S.jw);
                lds_barrier();
#pragma unroll
                for (int u = P / 2; u < P; ++u) v[u] = *reinterpret_cast<const V*>(lds + (sbr ^ N.su[u]));
#pragma unroll
                for (int u = 0; u < P / 2; ++u) v[u] = w[u];
                __builtin_amdgcn_s_setprio(0);
            }
        }
    }
}

}  // namespace tile
}  // namespace qsv
