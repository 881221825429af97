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

// Pair update of the pair kernels.  PK_DENSE: the 2x2 matvec of Algs. 1-2.
// Gates with more structure need less (Sec. 2.1 writes X, Y and Z out as
// such special cases): PK_ANTI, an anti-diagonal matrix [[0, u01], [u10, 0]]
// (Y and phased X): each output is one input times a phase, no sums;
// PK_SWAP, X itself: the pair is exchanged, data movement only (for a
// controlled X, Sec. 2.2's CNOT, half the pairs are exchanged).
enum { PK_DENSE = 0, PK_ANTI = 1, PK_SWAP = 2 };

template <typename R, typename V>
__device__ __forceinline__ V cmul_s(const V& a, R dr, R di) {
    V o;
    o.x = fmaR(-a.y, di, a.x * dr);
    o.y = fmaR(a.y, dr, a.x * di);
    return o;
}

template <typename R, int PK, typename V>
__device__ __forceinline__ void pair_op(const R* u, const V& a, const V& b, V& oa, V& ob) {
    if constexpr (PK == PK_DENSE) {
        mv2(u, a, b, oa, ob);
    } else if constexpr (PK == PK_ANTI) {
        oa = cmul_s(b, u[2], u[3]);
        ob = cmul_s(a, u[4], u[5]);
    } else {
        oa = b;
        ob = a;
    }
}

// ------------------------------------------------------------- Alg. 1
// Pair j -> a_j = insert0(j, p), b_j = a_j + 2^p; 2x2 matvec in place.
// CTRL: Alg. 2 with its control at a low index bit pc (below the 128-byte
// line): every pair over the target is read and written, and U applies
// where bit pc of a_j equals cs.  The pairs Alg. 2 would skip share lines
// with the ones it moves, so HBM carries the whole state either way; this
// form keeps every access a full, contiguous line.
template <typename R, bool CTRL = false, int PK = PK_DENSE>
__global__ __launch_bounds__(kThreads) void k_apply1q(typename V2T<R>::type* __restrict__ s,
                                                      uint64_t npairs, int p, M2<R> u, int pc = 0,
                                                      int cs = 0) {
    using V = typename V2T<R>::type;
    constexpr int P = GatePairs<R>::value;
    constexpr uint64_t BS = uint64_t(kThreads) * P;
    const BlockWalk bw(ceil_div(npairs, BS));
    for (uint64_t blk = bw.first; blk < bw.end; blk += bw.step) {
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
                pair_op<R, PK>(u.v, a[k], b[k], oa, ob);
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
template <typename R, int PK = PK_DENSE>
__global__ __launch_bounds__(kThreads) void k_applyc1q(typename V2T<R>::type* __restrict__ s,
                                                       uint64_t npairs, int plo, int phi, int pc,
                                                       int pt, int cs, M2<R> u) {
    using V = typename V2T<R>::type;
    constexpr int P = GatePairs<R>::value;
    constexpr uint64_t BS = uint64_t(kThreads) * P;
    const BlockWalk bw(ceil_div(npairs, BS));
    for (uint64_t blk = bw.first; blk < bw.end; blk += bw.step) {
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
                pair_op<R, PK>(u.v, a[k], b[k], oa, ob);
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
    const BlockWalk bw(ceil_div(nquads, BS));
    for (uint64_t blk = bw.first; blk < bw.end; blk += bw.step) {
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

// ------------------------------------------------ diagonal gates (one pass)
// A diagonal gate (Z, S, T, P, RZ, CZ, CP, ...) multiplies each amplitude by
// one entry of its diagonal and mixes nothing.  Item j names amplitude
//   x = j with zero bits inserted at positions f0 < f1 (nfix of them), then
//       the fixed bit values `fixval` set,
// which is multiplied by d[2 * bit(x, sa) + bit(x, sb)].  Fixing a bit
// restricts the pass to the amplitudes the gate changes: for P(theta) on
// position p, bit p = 1 (half the state); for a controlled phase, the
// control bit = cs and the target bit = 1 (a quarter).  With no fixed bits
// it is one linear pass over the state.
template <typename R>
struct D4 { R v[8]; };   // four complex entries (re, im)

template <typename R>
__global__ __launch_bounds__(kThreads) void k_diag(typename V2T<R>::type* __restrict__ s,
                                                   uint64_t items, int nfix, int f0, int f1,
                                                   uint64_t fixval, int sa, int sb, D4<R> d) {
    using V = typename V2T<R>::type;
    constexpr int P = PPT<R>::value;
    constexpr uint64_t BS = uint64_t(kThreads) * P;
    const BlockWalk bw(ceil_div(items, BS));
    for (uint64_t blk = bw.first; blk < bw.end; blk += bw.step) {
        const uint64_t j0 = blk * BS + threadIdx.x;
        V a[P];
        uint64_t xs[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint64_t j = j0 + uint64_t(k) * kThreads;
            uint64_t x = j;
            if (nfix > 0) x = insert0(x, f0);
            if (nfix > 1) x = insert0(x, f1);
            xs[k] = x | fixval;
            if (j < items) a[k] = ld_nt(s + xs[k]);
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint64_t j = j0 + uint64_t(k) * kThreads;
            if (j < items) {
                const int e = int(((xs[k] >> sa) & 1) * 2 + ((xs[k] >> sb) & 1));
                st_nt(s + xs[k], cmul_s(a[k], d.v[2 * e], d.v[2 * e + 1]));
            }
        }
    }
}

// ------------------------------------------- 2-qubit permutation (one pass)
// A 2-qubit gate whose matrix is a permutation with unit entries (SWAP of
// Sec. 2.3, CNOT written as a 4x4, ...) moves amplitudes and computes
// nothing.  For quad j (zero bits inserted at plo < phi) output element r
// (local index 2*x_qa + x_qb) takes input element src[r]; only the elements
// that move are read and written: SWAP touches two of the four.
struct Perm4 { int src[4]; };

template <typename R>
__global__ __launch_bounds__(kThreads) void k_perm2q(typename V2T<R>::type* __restrict__ s,
                                                     uint64_t nquads, int plo, int phi, int pa,
                                                     int pb, Perm4 pm) {
    using V = typename V2T<R>::type;
    const uint64_t wa = uint64_t(1) << pa, wb = uint64_t(1) << pb;
    const uint64_t off[4] = {0, wb, wa, wa + wb};
    const BlockWalk bw(ceil_div(nquads, kThreads));
    for (uint64_t blk = bw.first; blk < bw.end; blk += bw.step) {
        const uint64_t j = blk * kThreads + threadIdx.x;
        if (j >= nquads) continue;
        const uint64_t i0 = insert0(insert0(j, plo), phi);
        V v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (pm.src[r] != r) v[r] = ld_nt(s + i0 + off[pm.src[r]]);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (pm.src[r] != r) st_nt(s + i0 + off[r], v[r]);
    }
}

// ------------------------------------------- multi-controlled gates (Sec. 2.4)
// A gate with extra controls changes only the amplitudes whose control bits
// hold their values.  Item j names the first amplitude of one pair (NB = 1)
// or quad (NB = 2): j with a zero bit inserted at each of the npos positions
// of the controls and the gate's own bits (ascending, so each insertion
// leaves the lower ones in place -- Alg. 2's two insertions generalised),
// then the control values `fix` set.  Each control halves the items.
struct InsPos { int32_t p[kMaxQubits]; };

template <typename R, int NB, int PK = PK_DENSE>
__global__ __launch_bounds__(kThreads) void k_mc(typename V2T<R>::type* __restrict__ s,
                                                 uint64_t items, int npos, InsPos ip, uint64_t fix,
                                                 int pa, int pb, M4<R> u) {
    using V = typename V2T<R>::type;
    const uint64_t wa = uint64_t(1) << pa, wb = uint64_t(1) << pb;
    const BlockWalk bw(ceil_div(items, kThreads));
    for (uint64_t blk = bw.first; blk < bw.end; blk += bw.step) {
        const uint64_t j = blk * kThreads + threadIdx.x;
        if (j >= items) continue;
        uint64_t x = j;
        for (int i = 0; i < npos; ++i) x = insert0(x, ip.p[i]);
        x |= fix;
        if constexpr (NB == 1) {
            const V a = ld_nt(s + x), b = ld_nt(s + x + wa);
            V oa, ob;
            pair_op<R, PK>(u.v, a, b, oa, ob);
            st_nt(s + x, oa);
            st_nt(s + x + wa, ob);
        } else {
            // local index 2 * x_a + x_b (eq. (1) order of the 2-qubit gate)
            V in[4], out[4];
            in[0] = ld_nt(s + x);
            in[1] = ld_nt(s + x + wb);
            in[2] = ld_nt(s + x + wa);
            in[3] = ld_nt(s + x + wa + wb);
            mv4(u.v, in, out);
            st_nt(s + x, out[0]);
            st_nt(s + x + wb, out[1]);
            st_nt(s + x + wa, out[2]);
            st_nt(s + x + wa + wb, out[3]);
        }
    }
}

// ----------------------------------------- general k-qubit gate (Sec. 2.4)
// Item j: zero bits inserted at the k gate positions (ascending); slot c of
// the item is the amplitude at x + off[c], where off[c] spells the local
// index c over the gate's qubits in the caller's order.  Each thread loads
// its 2^K amplitudes, then forms and stores one output row at a time
// (row r = sum_c U[r][c] v[c]), so only the inputs stay in registers.  U
// sits in device memory and is read with uniform (scalar) loads.
template <int K>
struct KOff { uint64_t o[1 << K]; };

template <typename R, int K>
__global__ __launch_bounds__(kThreads) void k_kq(typename V2T<R>::type* __restrict__ s,
                                                 uint64_t items, InsPos ip, KOff<K> off,
                                                 const R* __restrict__ u) {
    using V = typename V2T<R>::type;
    constexpr int D = 1 << K;
    const BlockWalk bw(ceil_div(items, kThreads));
    for (uint64_t blk = bw.first; blk < bw.end; blk += bw.step) {
        const uint64_t j = blk * kThreads + threadIdx.x;
        if (j >= items) continue;
        uint64_t x = j;
#pragma unroll
        for (int i = 0; i < K; ++i) x = insert0(x, ip.p[i]);
        V v[D];
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = ld_nt(s + x + off.o[c]);
        // rows one at a time (not unrolled): the row index is uniform, so
        // the matrix row and the output offset come from scalar loads
#pragma unroll 1
        for (int r = 0; r < D; ++r) {
            R re, im;
            cmac_first(u[2 * D * r], u[2 * D * r + 1], v[0], re, im);
#pragma unroll
            for (int c = 1; c < D; ++c) cmac(u[2 * (D * r + c)], u[2 * (D * r + c) + 1], v[c], re, im);
            V o;
            o.x = re;
            o.y = im;
            st_nt(s + x + off.o[r], o);
        }
    }
}

// ------------------------------- dense k-qubit block on the matrix cores
// The gate of k_kq as real matrix products: with amplitudes split into
// (re, im), y = U x is a real product of the 2D x 2D matrix
// [[Re U, -Im U], [Im U, Re U]] (rows and columns interleaved per
// amplitude) with 2D x 16 real columns, 16 groups per wave.  One 16x16x4
// MFMA adds the product of a 16 x 4 slice of the matrix with a 4 x 16
// slice of the columns; D/2 of them give 16 output rows (8 amplitudes) of
// the 16 groups.  Lane l (group j = l mod 16, quarter q = l / 16) loads
// input amplitude 4m + q of its group whole and feeds its real part to
// slice 2m and its imaginary part to slice 2m + 1; it ends with amplitudes
// 8*rc + 2q and 8*rc + 2q + 1 of its group, both parts, for output slice
// rc.  The D/8 output slices accumulate side by side (independent chains
// for the matrix pipeline).  The host stores the matrix pre-arranged in
// this lane order (kq_mfma_pack), so the value a lane feeds to each
// product sits at a fixed index.  FP64 MFMA for complex128, FP32 MFMA for complex64: full
// precision, only the summation order differs from k_kq.  Needs 2^(n-K)
// to be a multiple of 64 (four waves of 16 groups per workgroup).
template <typename R>
struct MfmaOp;
template <>
struct MfmaOp<double> {
    typedef double acc __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct MfmaOp<float> {
    typedef float acc __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <typename R, int K>
__global__ __launch_bounds__(kThreads) void k_kq_mfma(typename V2T<R>::type* __restrict__ s,
                                                      uint64_t items, InsPos ip, KOff<K> off,
                                                      const R* __restrict__ apack) {
    using V = typename V2T<R>::type;
    using Acc = typename MfmaOp<R>::acc;
    constexpr int D = 1 << K;
    constexpr int NKC = D / 2;   // 4-row input slices
    constexpr int NRC = D / 8;   // 16-row output slices
    const int lane = int(threadIdx.x & 63u);
    const int wave = int(threadIdx.x >> 6);
    const int j = lane & 15, qq = lane >> 4;
    // the matrix in LDS, read at each product: held in registers (D^2/16 per
    // lane) it cost occupancy and measured slower for k = 4, 5
    __shared__ R alds[4 * D * D];
    for (int i = int(threadIdx.x); i < 4 * D * D; i += kThreads) alds[i] = apack[i];
    __syncthreads();
    const BlockWalk bw(items / 64);
    for (uint64_t blk = bw.first; blk < bw.end; blk += bw.step) {
        // keeps the LDS reads inside the loop (hoisted out of it, they would
        // hold every matrix value in registers again)
        asm volatile("" ::: "memory");
        uint64_t x = blk * 64 + uint64_t(wave) * 16 + uint64_t(j);
#pragma unroll
        for (int i = 0; i < K; ++i) x = insert0(x, ip.p[i]);
        R b[NKC];
#pragma unroll
        for (int m = 0; m < NKC / 2; ++m) {
            const V v = ld_nt(s + x + off.o[4 * m + qq]);
            b[2 * m] = v.x;
            b[2 * m + 1] = v.y;
        }
        Acc c[NRC];
#pragma unroll
        for (int rc = 0; rc < NRC; ++rc) c[rc] = Acc{R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
            for (int rc = 0; rc < NRC; ++rc)
                c[rc] = MfmaOp<R>::mma(alds[(rc * NKC + kc) * 64 + lane], b[kc], c[rc]);
#pragma unroll
        for (int rc = 0; rc < NRC; ++rc) {
            const int c0 = 8 * rc + 2 * qq;
            V o0, o1;
            o0.x = c[rc][0];
            o0.y = c[rc][1];
            o1.x = c[rc][2];
            o1.y = c[rc][3];
            st_nt(s + x + off.o[c0], o0);
            st_nt(s + x + off.o[c0 + 1], o1);
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

// ------------------------------------------------ structure of a gate matrix
// Exact tests on the FP64 entries (a complex64 state rounds them once, and
// 0 and 1 round to themselves).
inline bool czero(const double* u, int i) { return u[2 * i] == 0.0 && u[2 * i + 1] == 0.0; }
inline bool cone(const double* u, int i) { return u[2 * i] == 1.0 && u[2 * i + 1] == 0.0; }
inline bool is_diag2(const double* u) { return czero(u, 1) && czero(u, 2); }
inline bool is_anti2(const double* u) { return czero(u, 0) && czero(u, 3); }
inline bool is_x2(const double* u) { return is_anti2(u) && cone(u, 1) && cone(u, 2); }
inline bool is_diag4(const double* u) {
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            if (r != c && !czero(u, 4 * r + c)) return false;
    return true;
}
// A permutation matrix with unit entries: src[r] = the column of row r's 1.
inline bool is_perm4(const double* u, int* src) {
    int seen = 0;
    for (int r = 0; r < 4; ++r) {
        src[r] = -1;
        for (int c = 0; c < 4; ++c) {
            if (cone(u, 4 * r + c)) {
                if (src[r] >= 0) return false;
                src[r] = c;
            } else if (!czero(u, 4 * r + c)) {
                return false;
            }
        }
        if (src[r] < 0 || (seen >> src[r]) & 1) return false;
        seen |= 1 << src[r];
    }
    return true;
}

template <typename R>
constexpr int line_bits() { return sizeof(R) == 8 ? 3 : 4; }   // amplitudes per 128-byte line

// Launch k_diag over `items` amplitudes; d holds the four entries selected
// by 2 * bit(sa) + bit(sb) as (re, im) doubles.
template <typename R>
hipError_t diag_t(qsv_ctx ctx, void* s, uint64_t items, int nfix, int f0, int f1, uint64_t fixval,
                  int sa, int sb, const double* d) {
    using V = typename V2T<R>::type;
    D4<R> dd;
    for (int i = 0; i < 8; ++i) dd.v[i] = R(d[i]);
    prof_before(ctx, sizeof(R) == 8 ? "diag_c128" : "diag_c64", 2.0 * double(items) * sizeof(V));
    hipLaunchKernelGGL(k_diag<R>, dim3(grid_for<R>(items, PPT<R>::value)), dim3(kThreads), 0,
                       ctx->stream, static_cast<V*>(s), items, nfix, f0, f1, fixval, sa, sb, dd);
    prof_after(ctx);
    return hipGetLastError();
}

template <typename R>
hipError_t apply1q_t(qsv_ctx ctx, void* s, int n, int p, const double* u) {
    using V = typename V2T<R>::type;
    const uint64_t N = uint64_t(1) << n;
    const uint64_t np = N >> 1;
    if (is_diag2(u)) {
        // entries d0 (bit p = 0) and d1 (bit p = 1) at selector values 0 and 3
        const double d[8] = {u[0], u[1], 0, 0, 0, 0, u[6], u[7]};
        if (cone(u, 0) && p >= line_bits<R>())   // Z, S, T, P(theta): only bit p = 1 changes
            return diag_t<R>(ctx, s, np, 1, p, 0, uint64_t(1) << p, p, p, d);
        return diag_t<R>(ctx, s, N, 0, 0, 0, 0, p, p, d);
    }
    const bool anti = is_anti2(u), x = is_x2(u);
    prof_before(ctx, x ? (sizeof(R) == 8 ? "perm1q_c128" : "perm1q_c64")
                       : anti ? (sizeof(R) == 8 ? "anti1q_c128" : "anti1q_c64")
                              : (sizeof(R) == 8 ? "apply1q_c128" : "apply1q_c64"),
                2.0 * double(N) * sizeof(V));
    const dim3 grid(grid_for<R>(np, GatePairs<R>::value));
    if (x)
        hipLaunchKernelGGL((k_apply1q<R, false, PK_SWAP>), grid, dim3(kThreads), 0, ctx->stream,
                           static_cast<V*>(s), np, p, to_m2<R>(u), 0, 0);
    else if (anti)
        hipLaunchKernelGGL((k_apply1q<R, false, PK_ANTI>), grid, dim3(kThreads), 0, ctx->stream,
                           static_cast<V*>(s), np, p, to_m2<R>(u), 0, 0);
    else
        hipLaunchKernelGGL((k_apply1q<R, false>), grid, dim3(kThreads), 0, ctx->stream,
                           static_cast<V*>(s), np, p, to_m2<R>(u), 0, 0);
    prof_after(ctx);
    return hipGetLastError();
}

template <typename R>
hipError_t applyc1q_t(qsv_ctx ctx, void* s, int n, int pc, int pt, int cs, const double* u) {
    using V = typename V2T<R>::type;
    const uint64_t N = uint64_t(1) << n;
    const uint64_t np = N >> 2;
    const int plo = pc < pt ? pc : pt, phi = pc < pt ? pt : pc;
    const int lb = line_bits<R>();
    if (is_diag2(u)) {
        // U = diag(d0, d1) on the target where the control bit equals cs
        if (cone(u, 0) && pc >= lb && pt >= lb) {   // CZ, CP: a quarter of the state changes
            const double d[8] = {0, 0, 0, 0, 0, 0, u[6], u[7]};
            return diag_t<R>(ctx, s, np, 2, plo, phi, (uint64_t(cs) << pc) | (uint64_t(1) << pt), pt,
                             pt, d);
        }
        if (pc >= lb) {   // the half with the control bit set to cs
            const double d[8] = {u[0], u[1], 0, 0, 0, 0, u[6], u[7]};
            return diag_t<R>(ctx, s, 2 * np, 1, pc, 0, uint64_t(cs) << pc, pt, pt, d);
        }
        // control below the line: every line is touched; selector 2*c + t
        double d[8] = {1, 0, 1, 0, 1, 0, 1, 0};
        d[4 * cs + 0] = u[0];
        d[4 * cs + 1] = u[1];
        d[4 * cs + 2] = u[6];
        d[4 * cs + 3] = u[7];
        return diag_t<R>(ctx, s, N, 0, 0, 0, 0, pc, pt, d);
    }
    const bool anti = is_anti2(u), x = is_x2(u);
    prof_before(ctx, x ? (sizeof(R) == 8 ? "cperm1q_c128" : "cperm1q_c64")
                       : anti ? (sizeof(R) == 8 ? "canti1q_c128" : "canti1q_c64")
                              : (sizeof(R) == 8 ? "applyc1q_c128" : "applyc1q_c64"),
                double(N) * sizeof(V));
    // a control below the 128-byte line: the whole state moves anyway, so
    // move it in full lines (see k_apply1q)
    if (pc < lb) {
        const dim3 grid(grid_for<R>(2 * np, GatePairs<R>::value));
        if (x)
            hipLaunchKernelGGL((k_apply1q<R, true, PK_SWAP>), grid, dim3(kThreads), 0, ctx->stream,
                               static_cast<V*>(s), 2 * np, pt, to_m2<R>(u), pc, cs);
        else if (anti)
            hipLaunchKernelGGL((k_apply1q<R, true, PK_ANTI>), grid, dim3(kThreads), 0, ctx->stream,
                               static_cast<V*>(s), 2 * np, pt, to_m2<R>(u), pc, cs);
        else
            hipLaunchKernelGGL((k_apply1q<R, true>), grid, dim3(kThreads), 0, ctx->stream,
                               static_cast<V*>(s), 2 * np, pt, to_m2<R>(u), pc, cs);
    } else {
        const dim3 grid(grid_for<R>(np, GatePairs<R>::value));
        if (x)
            hipLaunchKernelGGL((k_applyc1q<R, PK_SWAP>), grid, dim3(kThreads), 0, ctx->stream,
                               static_cast<V*>(s), np, plo, phi, pc, pt, cs, to_m2<R>(u));
        else if (anti)
            hipLaunchKernelGGL((k_applyc1q<R, PK_ANTI>), grid, dim3(kThreads), 0, ctx->stream,
                               static_cast<V*>(s), np, plo, phi, pc, pt, cs, to_m2<R>(u));
        else
            hipLaunchKernelGGL((k_applyc1q<R>), grid, dim3(kThreads), 0, ctx->stream,
                               static_cast<V*>(s), np, plo, phi, pc, pt, cs, to_m2<R>(u));
    }
    prof_after(ctx);
    return hipGetLastError();
}

template <typename R>
hipError_t apply2q_t(qsv_ctx ctx, void* s, int n, int pa, int pb, const double* u) {
    using V = typename V2T<R>::type;
    const uint64_t N = uint64_t(1) << n;
    const uint64_t nq = N >> 2;
    const int plo = pa < pb ? pa : pb, phi = pa < pb ? pb : pa;
    const int lb = line_bits<R>();
    if (is_diag4(u)) {
        // entry r = 2*x_qa + x_qb of the diagonal, selected by bits (pa, pb)
        const double d[8] = {u[0], u[1], u[10], u[11], u[20], u[21], u[30], u[31]};
        if (cone(u, 0) && cone(u, 5) && cone(u, 10) && pa >= lb && pb >= lb)   // CZ, CP as a 4x4
            return diag_t<R>(ctx, s, nq, 2, plo, phi, (uint64_t(1) << pa) | (uint64_t(1) << pb), pa,
                             pb, d);
        return diag_t<R>(ctx, s, N, 0, 0, 0, 0, pa, pb, d);
    }
    Perm4 pm;
    if (is_perm4(u, pm.src)) {
        int moved = 0;
        for (int r = 0; r < 4; ++r) moved += pm.src[r] != r;
        prof_before(ctx, sizeof(R) == 8 ? "perm2q_c128" : "perm2q_c64",
                    2.0 * double(moved) * double(nq) * sizeof(V));
        hipLaunchKernelGGL(k_perm2q<R>, dim3(capped_grid((nq + kThreads - 1) / kThreads)), dim3(kThreads),
                           0, ctx->stream, static_cast<V*>(s), nq, plo, phi, pa, pb, pm);
        prof_after(ctx);
        return hipGetLastError();
    }
    prof_before(ctx, sizeof(R) == 8 ? "apply2q_c128" : "apply2q_c64", 2.0 * double(N) * sizeof(V));
    hipLaunchKernelGGL(k_apply2q<R>, dim3(grid_for<R>(nq, GateQuads<R>::value)), dim3(kThreads), 0,
                       ctx->stream, static_cast<V*>(s), nq, plo, phi, pa, pb, to_m4<R>(u));
    prof_after(ctx);
    return hipGetLastError();
}

// A gate with extra controls (PGate::cm / cv): a controlled 1q gate's own
// control joins them, so the base is U on one target or a 2-qubit U.
template <typename R>
hipError_t mc_t(qsv_ctx ctx, void* s, int n, const PGate& g) {
    using V = typename V2T<R>::type;
    uint64_t cm = g.cm, cv = g.cv;
    int nb = 1, pa = g.p0, pb = 0;
    if (g.kind == QSV_GC1Q) {
        cm |= uint64_t(1) << g.p0;
        if (g.cs) cv |= uint64_t(1) << g.p0;
        pa = g.p1;
    } else if (g.kind == QSV_G2Q) {
        nb = 2;
        pb = g.p1;
    }
    const uint64_t ins = cm | (uint64_t(1) << pa) | (nb == 2 ? uint64_t(1) << pb : 0);
    InsPos ip{};
    int npos = 0;
    for (int p = 0; p < n; ++p)
        if ((ins >> p) & 1) ip.p[npos++] = p;
    const uint64_t items = uint64_t(1) << (n - npos);
    M4<R> u{};
    for (int i = 0; i < (nb == 2 ? 32 : 8); ++i) u.v[i] = R(g.m[i]);
    const dim3 grid(capped_grid((items + kThreads - 1) / kThreads));
    const double bytes = 2.0 * double(items << nb) * sizeof(V);
    if (nb == 2) {
        prof_before(ctx, sizeof(R) == 8 ? "mc2q_c128" : "mc2q_c64", bytes);
        hipLaunchKernelGGL((k_mc<R, 2>), grid, dim3(kThreads), 0, ctx->stream, static_cast<V*>(s), items,
                           npos, ip, cv, pa, pb, u);
    } else if (is_x2(g.m)) {   // Toffoli and other multi-controlled X: the pairs swap
        prof_before(ctx, sizeof(R) == 8 ? "mcx_c128" : "mcx_c64", bytes);
        hipLaunchKernelGGL((k_mc<R, 1, PK_SWAP>), grid, dim3(kThreads), 0, ctx->stream, static_cast<V*>(s),
                           items, npos, ip, cv, pa, pb, u);
    } else {
        prof_before(ctx, sizeof(R) == 8 ? "mc1q_c128" : "mc1q_c64", bytes);
        hipLaunchKernelGGL((k_mc<R, 1>), grid, dim3(kThreads), 0, ctx->stream, static_cast<V*>(s), items,
                           npos, ip, cv, pa, pb, u);
    }
    prof_after(ctx);
    return hipGetLastError();
}

// k-qubit gate: positions pos[i] of the caller's qubits (pos[0] = most
// significant local bit), U already in device memory in the state's type.
template <typename R, int K>
hipError_t kq_launch(qsv_ctx ctx, void* s, int n, const int* pos, const void* du, bool mfma) {
    using V = typename V2T<R>::type;
    InsPos ip{};
    int sorted[K];
    for (int i = 0; i < K; ++i) sorted[i] = pos[i];
    for (int i = 1; i < K; ++i)
        for (int j = i; j > 0 && sorted[j - 1] > sorted[j]; --j) std::swap(sorted[j - 1], sorted[j]);
    for (int i = 0; i < K; ++i) ip.p[i] = sorted[i];
    KOff<K> off{};
    for (int c = 0; c < (1 << K); ++c) {
        uint64_t o = 0;
        for (int i = 0; i < K; ++i)
            if ((c >> (K - 1 - i)) & 1) o |= uint64_t(1) << pos[i];
        off.o[c] = o;
    }
    const uint64_t items = uint64_t(1) << (n - K);
    if constexpr (K >= 3) {
        if (mfma) {
            if (items % 64 != 0) return hipErrorInvalidValue;   // the caller checks kq_mfma_applies
            prof_before(ctx, sizeof(R) == 8 ? "kq_mfma_c128" : "kq_mfma_c64",
                        2.0 * double(uint64_t(1) << n) * sizeof(V));
            hipLaunchKernelGGL((k_kq_mfma<R, K>), dim3(capped_grid(items / 64)), dim3(kThreads), 0, ctx->stream,
                               static_cast<V*>(s), items, ip, off, static_cast<const R*>(du));
            const hipError_t e = hipGetLastError();
            prof_after(ctx);
            return e;
        }
    }
    if (mfma) return hipErrorInvalidValue;
    prof_before(ctx, sizeof(R) == 8 ? "kq_c128" : "kq_c64", 2.0 * double(uint64_t(1) << n) * sizeof(V));
    hipLaunchKernelGGL((k_kq<R, K>), dim3(capped_grid((items + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       ctx->stream, static_cast<V*>(s), items, ip, off, static_cast<const R*>(du));
    prof_after(ctx);
    return hipGetLastError();
}

template <typename R>
hipError_t kq_t(qsv_ctx ctx, void* s, int n, int k, const int* pos, const void* du, bool mfma) {
    switch (k) {
    case 1: return kq_launch<R, 1>(ctx, s, n, pos, du, mfma);
    case 2: return kq_launch<R, 2>(ctx, s, n, pos, du, mfma);
    case 3: return kq_launch<R, 3>(ctx, s, n, pos, du, mfma);
    case 4: return kq_launch<R, 4>(ctx, s, n, pos, du, mfma);
    case 5: return kq_launch<R, 5>(ctx, s, n, pos, du, mfma);
    default: return hipErrorInvalidValue;
    }
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
hipError_t launch_kq(qsv_ctx ctx, void* s, int n, int dtype, int k, const int* pos, const void* du, bool mfma) {
    return dtype == QSV_C128 ? kq_t<double>(ctx, s, n, k, pos, du, mfma)
                             : kq_t<float>(ctx, s, n, k, pos, du, mfma);
}
bool kq_mfma_applies(int n, int k, int mode) {
    if (n - k < 6) return false;
    // mode 1: where the matrix cores measured faster than the vector kernel
    // (k = 3, 5; for k = 4 both run near the HBM rate and the vector kernel
    // was slightly ahead); mode 2: every k in 3..5
    return mode == 2 ? (k >= 3 && k <= 5) : mode == 1 ? (k == 3 || k == 5) : false;
}
void kq_mfma_pack(int dtype, int k, const double* u, void* out) {
    const int D = 1 << k;
    for (int rc = 0; rc < D / 8; ++rc)
        for (int kc = 0; kc < D / 2; ++kc)
            for (int lane = 0; lane < 64; ++lane) {
                // A[i][kk] of the 16x16x4 MFMA sits on lane i + 16 kk; output
                // row i of a slice is element i / 4 of lane group i mod 4 for
                // the FP64 instruction and element i mod 4 of group i / 4 for
                // the FP32 one
                const int i = lane & 15, kk = lane >> 4;
                const int g = dtype == QSV_C128 ? i % 4 : i / 4;
                const int e = dtype == QSV_C128 ? i / 4 : i % 4;
                const int co = 8 * rc + 2 * g + e / 2, po = e % 2;
                const int ci = 4 * (kc / 2) + kk, pi = kc % 2;
                const double re = u[2 * (co * D + ci)], im = u[2 * (co * D + ci) + 1];
                // [[Re U, -Im U], [Im U, Re U]], rows and columns (re, im) per amplitude
                const double v = po == 0 ? (pi == 0 ? re : -im) : (pi == 0 ? im : re);
                const size_t at = size_t(rc * (D / 2) + kc) * 64 + size_t(lane);
                if (dtype == QSV_C128) static_cast<double*>(out)[at] = v;
                else static_cast<float*>(out)[at] = float(v);
            }
}
hipError_t launch_gate(qsv_ctx ctx, void* s, int n, int dtype, const PGate& g) {
    if (g.cm) return dtype == QSV_C128 ? mc_t<double>(ctx, s, n, g) : mc_t<float>(ctx, s, n, g);
    switch (g.kind) {
    case QSV_G1Q: return launch_apply1q(ctx, s, n, dtype, g.p0, g.m);
    case QSV_GC1Q: return launch_applyc1q(ctx, s, n, dtype, g.p0, g.p1, g.cs, g.m);
    case QSV_G2Q: return launch_apply2q(ctx, s, n, dtype, g.p0, g.p1, g.m);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qsv
