// Adjoint-method gradient sweep (Jones & Gacon, arXiv:2009.02823) over the
// gate engine: lambda = O psi, then for k = last..first
//   rotation exp(-i theta P/2):  g_k = Im <lambda| P |psi>
//   psi <- U_k^dag psi,  lambda <- U_k^dag lambda.
// Fused form (default): the reversed, daggered circuit is grouped into tile
// passes over both vectors.  Inside a pass each rotation stays a separate
// gate: its partial Im<lam|P|psi> over the tile is taken in registers right
// before the rotation is rewound, reduced across each wave in a fixed
// butterfly order and stored per (tile, wave, slot); a second kernel adds
// them in a fixed order.  Every other gate may be fused as in the forward
// passes.  Unfused form: one kernel per gate, each rotation's partial fused
// into its rewind pass.  All gradients come back to the host in one copy.
#include <cstring>

#include "qsv_tile_core.h"

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
    for (uint64_t x = uint64_t(blockIdx.x) * kThreads + threadIdx.x; x < N;
         x += uint64_t(gridDim.x) * kThreads) {
        double d = 0.0;
        for (int t = 0; t < nt; ++t) d += (__popcll(x & masks[t]) & 1) ? -w[t] : w[t];
        const V v = psi[x];
        V o;
        o.x = R(d * double(v.x));
        o.y = R(d * double(v.y));
        lam[x] = o;
    }
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

// ------------------------------------------------- two-vector tile passes
using namespace tile;

template <int B, int AXIS, typename V, int P>
__device__ __forceinline__ double rot_part(const V (&v)[P], const V (&l)[P]) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (!(i & (1 << B))) {
            const int j = i | (1 << B);
            const double ar = v[i].x, ai = v[i].y, br = v[j].x, bi = v[j].y;
            double qar, qai, qbr, qbi;   // (P psi)_i, (P psi)_j
            if (AXIS == QSV_AXIS_X) {
                qar = br; qai = bi; qbr = ar; qbi = ai;
            } else if (AXIS == QSV_AXIS_Y) {
                qar = bi; qai = -br; qbr = -ai; qbi = ar;
            } else {
                qar = ar; qai = ai; qbr = -br; qbi = -bi;
            }
            acc += double(l[i].x) * qai - double(l[i].y) * qar + double(l[j].x) * qbi -
                   double(l[j].y) * qbr;
        }
    return acc;
}

// Sum of a double over the 64 lanes of a wave with DPP lane moves (no LDS
// traffic, short dependent latency); the total lands in lane 63.  Lanes a
// move reads from outside the row, or rows the row mask leaves out, add 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWS, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_to_lane63(double s) {
    s += dpp_move<0x111, 0xf>(s);   // row_shr:1
    s += dpp_move<0x112, 0xf>(s);   // row_shr:2
    s += dpp_move<0x114, 0xf>(s);   // row_shr:4
    s += dpp_move<0x118, 0xf>(s);   // row_shr:8: lane 15 of each row holds the row sum
    s += dpp_move<0x142, 0xa>(s);   // row_bcast:15 into rows 1 and 3
    s += dpp_move<0x143, 0xc>(s);   // row_bcast:31 into rows 2 and 3
    return s;
}

// The gate on both vectors, in place; a rotation also emits its partial
// Im<lam|P|psi> (taken before the rotation is undone).  SPEC selects the
// rotation bodies that use the structure of the axis.
template <int RB, bool SPEC, typename R, typename V, int P>
__device__ __forceinline__ void apply_gate2(V (&v)[P], V (&l)[P], const TGate<R>& g,
                                            double* __restrict__ part_out, uint32_t tid) {
    if (g.kind == DK_ROT) {
        double part = 0.0;
        on_bit<RB>(g.r0, [&](auto B) __attribute__((always_inline)) {
            constexpr int b = decltype(B)::value;
            // the rewind exp(+i theta P / 2) has the structure of its axis:
            // X -> [[c, i s], [i s, c]], Y -> real, Z -> diagonal
            if constexpr (!SPEC) {
                if (g.cs == QSV_AXIS_X) part = rot_part<b, QSV_AXIS_X>(v, l);
                else if (g.cs == QSV_AXIS_Y) part = rot_part<b, QSV_AXIS_Y>(v, l);
                else part = rot_part<b, QSV_AXIS_Z>(v, l);
                rg_1q<b>(v, v, g.m);
                rg_1q<b>(l, l, g.m);
            } else if (g.cs == QSV_AXIS_X) {
                part = rot_part<b, QSV_AXIS_X>(v, l);
                rg_1x<b>(v, v, g.m);
                rg_1x<b>(l, l, g.m);
            } else if (g.cs == QSV_AXIS_Y) {
                part = rot_part<b, QSV_AXIS_Y>(v, l);
                rg_1r<b>(v, v, g.m);
                rg_1r<b>(l, l, g.m);
            } else {
                part = rot_part<b, QSV_AXIS_Z>(v, l);
                rg_1d<b>(v, v, g.m + 8);
                rg_1d<b>(l, l, g.m + 8);
            }
        });
        part = wave_sum_to_lane63(part);
        if ((tid & 63) == 63) part_out[size_t(g.r1) * gridDim.x * 4 + (tid >> 6)] = part;
    } else {
        apply_op2_inplace<RB>(v, l, g.kind * 64 + g.r0 * 8 + g.r1, g.m);
    }
}

// One two-vector tile pass.  partials: this pass's block of
// [slot][tile][wave] doubles (slot count in the header's pad field), so the
// per-rotation sums read each slot's row contiguously.
// SPLIT: consecutive stages share a register bit and each vector changes
// mapping in two half-tile rounds through LDS (see run_stages), so the two
// tiles take half the LDS.
template <typename R, int K, bool SPLIT, bool SPEC>
__global__ __launch_bounds__(kThreads) void k_adj_tile(typename V2T<R>::type* __restrict__ psi,
                                                       typename V2T<R>::type* __restrict__ lam,
                                                       const char* __restrict__ plan,
                                                       double* __restrict__ partials) {
    using V = typename V2T<R>::type;
    constexpr int E = SPLIT ? 1 << (K - 1) : 1 << K;   // LDS amplitudes per vector
    constexpr int RB = K - 8;
    constexpr int P = 1 << RB;
    constexpr uint32_t ES = sizeof(V);
    __shared__ V tp[E];
    __shared__ V tl[E];
    char* lp = reinterpret_cast<char*>(tp);
    char* ll = reinterpret_cast<char*>(tl);

    const TPassHdr* hdr = reinterpret_cast<const TPassHdr*>(plan);
    const TStage* stg = reinterpret_cast<const TStage*>(plan + sizeof(TPassHdr));
    const int nst = hdr->nstages;
    const TGate<R>* gates = reinterpret_cast<const TGate<R>*>(plan + sizeof(TPassHdr) +
                                                              size_t(nst) * sizeof(TStage));
    const uint32_t tid = threadIdx.x;
    double* const part_out = partials + size_t(blockIdx.x) * 4;

    uint64_t b = blockIdx.x;
#pragma unroll
    for (int i = 0; i < K; ++i) b = insert0(b, hdr->pos[i]);
    const uint64_t xt = b | deposit(tid, hdr->tpos_ld, 8);
    V* const sp = psi + xt;
    V* const sl = lam + xt;
    V v[P], l[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
        v[u] = ld_nt(sp + hdr->du[u]);
        l[u] = ld_nt(sl + hdr->du[u]);
    }
    for (int st = 0; st < nst; ++st) {
        const TStage& S = stg[st];
        const uint32_t sb = swz<R>(deposit32(tid, S.tbits, 8)) * ES;
        if (!SPLIT && st > 0) {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                v[u] = *reinterpret_cast<const V*>(lp + (sb ^ S.su[u]));
                l[u] = *reinterpret_cast<const V*>(ll + (sb ^ S.su[u]));
            }
        }
        // in place: two register sets per vector (as in the one-state
        // kernel) would double the registers and halve the occupancy
        for (int g = S.gbeg; g < S.gend; ++g) apply_gate2<RB, SPEC>(v, l, gates[g], part_out, tid);
        if (!SPLIT && st < nst - 1) {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                *reinterpret_cast<V*>(lp + (sb ^ S.su_wr[u])) = v[u];
                *reinterpret_cast<V*>(ll + (sb ^ S.su_wr[u])) = l[u];
            }
            lds_barrier();
        }
        if (SPLIT && st < nst - 1) {
            const TStage& N = stg[st + 1];
            const uint32_t sbw = swz<R>(deposit32(tid, S.tbw, 8)) * ES;
            const uint32_t sbr = swz<R>(deposit32(tid, N.tbr, 8)) * ES;
            V wv[P / 2], wl[P / 2];
            if (st > 0) lds_barrier();   // the previous change's reads are done
            write_half<RB, 0>(v, lp, sbw, S.su_wr, S.jw);
            write_half<RB, 0>(l, ll, sbw, S.su_wr, S.jw);
            lds_barrier();
#pragma unroll
            for (int u = 0; u < P / 2; ++u) {
                wv[u] = *reinterpret_cast<const V*>(lp + (sbr ^ N.su[u]));
                wl[u] = *reinterpret_cast<const V*>(ll + (sbr ^ N.su[u]));
            }
            lds_barrier();
            write_half<RB, 1>(v, lp, sbw, S.su_wr, S.jw);
            write_half<RB, 1>(l, ll, sbw, S.su_wr, S.jw);
            lds_barrier();
#pragma unroll
            for (int u = P / 2; u < P; ++u) {
                v[u] = *reinterpret_cast<const V*>(lp + (sbr ^ N.su[u]));
                l[u] = *reinterpret_cast<const V*>(ll + (sbr ^ N.su[u]));
            }
#pragma unroll
            for (int u = 0; u < P / 2; ++u) {
                v[u] = wv[u];
                l[u] = wl[u];
            }
        }
    }
    const uint64_t xs = b | deposit(tid, hdr->tpos_st, 8);
    V* const sq = psi + xs;
    V* const sm = lam + xs;
#pragma unroll
    for (int u = 0; u < P; ++u) {
        st_nt(sq + hdr->du_st[u], v[u]);
        st_nt(sm + hdr->du_st[u], l[u]);
    }
}

// grad[tag[s]] = sum over (tile, wave) of partials[(s * tiles + tile) * 4 + wave], fixed order
__global__ __launch_bounds__(kThreads) void k_adj_cols(const double* __restrict__ partials,
                                                       int tiles, int nslot,
                                                       const int32_t* __restrict__ tags,
                                                       double* __restrict__ grad) {
    __shared__ double red[1][kThreads];
    const int s = blockIdx.x;
    double acc = 0.0;
    for (int t = threadIdx.x; t < tiles; t += kThreads) {
        const double* p = partials + (size_t(s) * tiles + t) * 4;
        acc += (p[0] + p[1]) + (p[2] + p[3]);
    }
    red[0][threadIdx.x] = acc;
    double tot[1];
    block_tree256<1>(red, tot);
    if (threadIdx.x == 0) grad[tags[s]] = tot[0];
}

// Two-vector tile shape per precision (measured on a 24-qubit, 480-angle
// circuit): 2^11 amplitudes with split exchange for both.  complex128: 32 KiB
// of LDS and about 135 registers, three workgroups per CU.  complex64: 16 KiB
// and about 100 registers with the generic 2x2 rotation body, four waves per
// SIMD; the axis-specialised bodies take it to 132 registers (three waves)
// and 2^12 tiles with full exchange to 200 (two), both slower (adjoint sweep
// 9.67 and 9.88 ms against 9.50).
template <typename R>
struct AdjShape {
    static constexpr int K = 11;
    static constexpr bool SPLIT = true;
    static constexpr bool SPEC = sizeof(R) == 8;
};

template <typename R>
hipError_t launch_adj_tile(qsv_ctx ctx, void* psi, void* lam, int n, const char* rec,
                           double* partials) {
    using V = typename V2T<R>::type;
    using S = AdjShape<R>;
    const unsigned tiles = unsigned(uint64_t(1) << (n - S::K));
    hipLaunchKernelGGL((k_adj_tile<R, S::K, S::SPLIT, S::SPEC>), dim3(tiles), dim3(kThreads), 0,
                       ctx->stream, static_cast<V*>(psi), static_cast<V*>(lam), rec, partials);
    return hipGetLastError();
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
hipError_t rewind_one(qsv_ctx ctx, void* psi, void* lam, int n, const PGate& g, int axis,
                      double* dgrad_slot) {
    using V = typename V2T<R>::type;
    const int dt = sizeof(R) == 8 ? QSV_C128 : QSV_C64;
    const uint64_t N = uint64_t(1) << n;
    PGate d;
    dagger(g, d);
    if (axis < 0) {
        hipError_t e = launch_gate(ctx, psi, n, dt, d);
        if (e != hipSuccess) return e;
        return launch_gate(ctx, lam, n, dt, d);
    }
    const uint64_t npairs = N / 2;
    const unsigned G = adj_blocks(npairs);
    const uint64_t chunk = (npairs + G - 1) / G;
    M2<R> ud;
    for (int i = 0; i < 8; ++i) ud.v[i] = R(d.m[i]);
    prof_before(ctx, sizeof(R) == 8 ? "adj_rot_c128" : "adj_rot_c64", 4.0 * double(N) * sizeof(V));
    switch (axis) {
    case QSV_AXIS_X:
        hipLaunchKernelGGL((k_adj_rot<R, QSV_AXIS_X>), dim3(G), dim3(kThreads), 0, ctx->stream,
                           static_cast<V*>(psi), static_cast<V*>(lam), npairs, chunk, g.p0, ud,
                           ctx->d_red);
        break;
    case QSV_AXIS_Y:
        hipLaunchKernelGGL((k_adj_rot<R, QSV_AXIS_Y>), dim3(G), dim3(kThreads), 0, ctx->stream,
                           static_cast<V*>(psi), static_cast<V*>(lam), npairs, chunk, g.p0, ud,
                           ctx->d_red);
        break;
    default:
        hipLaunchKernelGGL((k_adj_rot<R, QSV_AXIS_Z>), dim3(G), dim3(kThreads), 0, ctx->stream,
                           static_cast<V*>(psi), static_cast<V*>(lam), npairs, chunk, g.p0, ud,
                           ctx->d_red);
        break;
    }
    prof_after(ctx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(kThreads), 0, ctx->stream, ctx->d_red, int(G),
                       dgrad_slot);
    return hipGetLastError();
}

template <typename R>
hipError_t adjoint_t(qsv_ctx ctx, void* psi, void* lam, int n, const std::vector<PGate>& fwd,
                     const std::vector<int>& rot_param, const std::vector<int>& rot_axis,
                     int nterms, const uint64_t* pmasks, const double* w, double* grad_by_gate,
                     bool fused) {
    using V = typename V2T<R>::type;
    const int dt = sizeof(R) == 8 ? QSV_C128 : QSV_C64;
    const uint64_t N = uint64_t(1) << n;
    const size_t ng = fwd.size();
    constexpr int KA = AdjShape<R>::K;
    if (n < KA || n - KA > kMaxTileGridLog2) fused = false;   // too small, or too many tiles for one launch

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
    prof_before(ctx, sizeof(R) == 8 ? "adj_obs_c128" : "adj_obs_c64", 2.0 * double(N) * sizeof(V));
    hipLaunchKernelGGL(k_apply_obs<R>, dim3(capped_grid((N + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, ctx->stream, static_cast<const V*>(psi), static_cast<V*>(lam), N, nterms,
                       dmask, dw);
    prof_after(ctx);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    bool any_rot = false;
    for (size_t kk = 0; kk < ng; ++kk) any_rot |= rot_param[kk] >= 0;

    if (!fused) {
        e = ensure_aux(ctx, ng + 1);
        if (e != hipSuccess) return e;
        for (size_t kk = ng; kk-- > 0;) {
            e = rewind_one<R>(ctx, psi, lam, n, fwd[kk], rot_param[kk] >= 0 ? rot_axis[kk] : -1,
                              ctx->d_aux + kk);
            if (e != hipSuccess) return e;
        }
    } else {
        // the reversed, daggered circuit; rotations kept as KROT with their forward index
        std::vector<PGate> rev;
        rev.reserve(ng);
        for (size_t kk = ng; kk-- > 0;) {
            PGate d;
            dagger(fwd[kk], d);
            if (rot_param[kk] >= 0) {
                d.kind = KROT;
                d.cs = rot_axis[kk];
                d.tag = int(kk);
            }
            rev.push_back(d);
        }
        rev = prefuse(rev);
        // same structure as the last sweep (new angles): same passes
        const std::vector<Pass>& passes =
            plan_memo(ctx->adj_memo, n, rev,
                      TileConfig{KA, sizeof(R) == 8 ? 3 : 4, KA - 8, coal_bits_for(dt),
                                 AdjShape<R>::SPLIT ? 1 : 0});
        // slots, record layout, partial-buffer size
        size_t bytes = 0, max_part = 0;
        std::vector<size_t> offs(passes.size(), 0), tag_off(passes.size(), 0);
        std::vector<int> nslot(passes.size(), 0);
        for (size_t i = 0; i < passes.size(); ++i) {
            const Pass& ps = passes[i];
            if (ps.single) continue;
            int s = 0;
            for (int gi : ps.gates)
                if (rev[size_t(gi)].kind == KROT) rev[size_t(gi)].p1 = s++;
            nslot[i] = s;
            offs[i] = bytes;
            bytes += pass_record_bytes(dt, ps);
            tag_off[i] = bytes;
            bytes += (size_t(s) * sizeof(int32_t) + 255) & ~size_t(255);
            const size_t part = (size_t(1) << (n - KA)) * size_t(s) * 4;
            if (part > max_part) max_part = part;
        }
        e = ensure_aux(ctx, ng + 1 + max_part);
        if (e != hipSuccess) return e;
        double* dgrad = ctx->d_aux;
        double* dpart = ctx->d_aux + ng + 1;
        char* drec = nullptr;
        if (bytes) {
            e = plan_staging(ctx, bytes, &host);
            if (e != hipSuccess) return e;
            char* h = static_cast<char*>(host);
            for (size_t i = 0; i < passes.size(); ++i) {
                const Pass& ps = passes[i];
                if (ps.single) continue;
                if (!write_pass_record(dt, h + offs[i], rev, ps)) return hipErrorInvalidValue;
                reinterpret_cast<TPassHdr*>(h + offs[i])->pad = nslot[i];
                int32_t* tags = reinterpret_cast<int32_t*>(h + tag_off[i]);
                for (int gi : ps.gates)
                    if (rev[size_t(gi)].kind == KROT) tags[rev[size_t(gi)].p1] = rev[size_t(gi)].tag;
            }
            e = plan_upload(ctx, bytes, &dev);
            if (e != hipSuccess) return e;
            drec = static_cast<char*>(dev);
        }
        const int tiles = int(uint64_t(1) << (n - KA));
        for (size_t i = 0; i < passes.size(); ++i) {
            const Pass& ps = passes[i];
            if (ps.single) {
                const PGate& g = rev[size_t(ps.gates[0])];
                if (g.kind == KROT) {
                    // rewind_one daggers its argument: hand it the forward gate
                    e = rewind_one<R>(ctx, psi, lam, n, fwd[size_t(g.tag)], g.cs, dgrad + g.tag);
                } else {
                    e = launch_gate(ctx, psi, n, dt, g);
                    if (e == hipSuccess) e = launch_gate(ctx, lam, n, dt, g);
                }
                if (e != hipSuccess) return e;
                continue;
            }
            prof_before(ctx, sizeof(R) == 8 ? "adj_tile_c128" : "adj_tile_c64",
                        4.0 * double(N) * sizeof(V));
            e = launch_adj_tile<R>(ctx, psi, lam, n, drec + offs[i], dpart);
            prof_after(ctx);
            if (e != hipSuccess) return e;
            if (nslot[i] > 0) {
                hipLaunchKernelGGL(k_adj_cols, dim3(unsigned(nslot[i])), dim3(kThreads), 0,
                                   ctx->stream, dpart, tiles, nslot[i],
                                   reinterpret_cast<const int32_t*>(drec + tag_off[i]), dgrad);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
        }
    }
    for (size_t kk = 0; kk < ng; ++kk) grad_by_gate[kk] = 0.0;
    if (any_rot) {
        std::vector<double> tmp(ng, 0.0);
        e = hipMemcpyAsync(tmp.data(), ctx->d_aux, ng * sizeof(double), hipMemcpyDeviceToHost,
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
                       const double* w, double* grad_by_gate, bool fused) {
    return dtype == QSV_C128
               ? adjoint_t<double>(ctx, psi, lam, n, fwd, rot_param, rot_axis, nterms, pmasks, w,
                                   grad_by_gate, fused)
               : adjoint_t<float>(ctx, psi, lam, n, fwd, rot_param, rot_axis, nterms, pmasks, w,
                                  grad_by_gate, fused);
}

}  // namespace qsv
