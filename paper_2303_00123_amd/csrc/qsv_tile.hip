// Fused tile pass.
//
// One workgroup of 256 threads owns a tile of 2^K amplitudes spanning the
// pass's K index-bit positions: tile t covers the indices whose non-tile
// bits spell t (zero-bit insertion at each tile position, ascending -- the
// masks of Sec. 2.1-2.2 generalised from one or two positions to K).  The
// tile positions always include the lowest bits, so a tile is a set of
// contiguous runs and the loads and stores stay coalesced.
//
// Each thread holds P = 2^(K-8) amplitudes in registers.  A gate whose bits
// are all register bits is applied without leaving registers, with the
// pair/quad index maps of Algs. 1-3 resolved at compile time (one code path
// per register-bit choice).  Between stages the tile is re-mapped through
// LDS, so different local bits become register bits.  HBM sees one read and
// one write of the tile for the whole gate group.
//
// LDS holds the tile with an XOR swizzle on the 16-byte (c128) or 8-byte
// (c64) slot index, so strided stage mappings spread over the banks.
#include <array>
#include <cstdlib>
#include <vector>

#include "qsv_tile_core.h"

namespace qsv {
namespace {

using namespace tile;

// ------------------------------------------------------------ the kernel
// One workgroup per tile.  Every stage record (including the first and the
// last, which carry the load mapping) drives the same loop body, so the gate
// dispatch is compiled once.  Slot offsets come precomputed in the plan.
template <typename R, int K, int RB, bool SPLIT>
__global__ __launch_bounds__(1 << (K - RB)) void k_tile(typename V2T<R>::type* __restrict__ s,
                                                        const char* __restrict__ plan, int from_zero) {
    using V = typename V2T<R>::type;
    constexpr int E = SPLIT ? 1 << (K - 1) : 1 << K;   // LDS amplitudes
    constexpr int TB = K - RB;
    constexpr int P = 1 << RB;
    __shared__ V tile[E];
    char* lds = reinterpret_cast<char*>(tile);

    const TPassHdr* hdr = reinterpret_cast<const TPassHdr*>(plan);
    const TStage* stg = reinterpret_cast<const TStage*>(plan + sizeof(TPassHdr));
    const int nst = hdr->nstages;
    const TGate<R>* gates = reinterpret_cast<const TGate<R>*>(plan + sizeof(TPassHdr) +
                                                              size_t(nst) * sizeof(TStage));
    const uint32_t tid = threadIdx.x;

    // Tile of this workgroup.  Workgroups go to the 8 XCDs round-robin
    // (block b on XCD b % 8); give each XCD a contiguous run of tiles in
    // dispatch order, so tiles that differ only in the lowest non-tile bits
    // (which share 128-byte lines when the tile keeps fewer than 3 or 4 low
    // bits) are resident together on one XCD and meet in its L2.
    const uint32_t ntiles = gridDim.x;
    uint64_t b = blockIdx.x;
    if ((ntiles & 7u) == 0) b = (blockIdx.x & 7u) * (ntiles >> 3) + (blockIdx.x >> 3);
    // per-thread pointer to this tile's slot-0 amplitude; slot u adds the
    // uniform offset du[u] (disjoint bits, so OR == ADD)
#pragma unroll
    for (int i = 0; i < K; ++i) b = insert0(b, hdr->pos[i]);
    const uint64_t xt = b | deposit(tid, hdr->tpos_ld, TB);
    V* const sp = s + xt;

    // memory and LDS phases run at raised wave priority, so the other
    // resident workgroup's arithmetic fills the gaps instead of delaying them
    V v[P];
    __builtin_amdgcn_s_setprio(2);
    if (from_zero) {
        // the circuit starts from |0...0>: the first pass makes it in
        // registers (amplitude 1 at index 0) instead of reading the state
#pragma unroll
        for (int u = 0; u < P; ++u) {
            v[u].x = (xt | hdr->du[u]) == 0 ? R(1) : R(0);
            v[u].y = R(0);
        }
    } else {
#pragma unroll
        for (int u = 0; u < P; ++u) v[u] = ld_nt(sp + hdr->du[u]);
    }
    __builtin_amdgcn_s_setprio(0);
    run_stages<R, K, RB, SPLIT>(v, lds, stg, nst, gates, tid);
    V* const sq = s + (b | deposit(tid, hdr->tpos_st, TB));
    __builtin_amdgcn_s_setprio(2);
#pragma unroll
    for (int u = 0; u < P; ++u) st_nt(sq + hdr->du_st[u], v[u]);
}

// ------------------------------------------------------------ host side
bool is_zero(double x) { return x == 0.0; }


// Lower a host gate to the device record of its stage.  Returns false if a
// gate bit is not a register bit of the stage (a planner bug).
template <typename R>
bool to_device_gate(const PGate& g, const int* loc, const Stage& st, TGate<R>& t) {
    if (g.cm) return false;   // extra controls never reach a tile pass
    int reg[32];
    for (int b = 0; b < 32; ++b) reg[b] = -1;
    for (int j = 0; j < st.nr; ++j) reg[st.rbits[j]] = j;
    for (int m = 0; m < 32; ++m) t.m[m] = R(0);
    t.cs = 1;
    if (loc[g.p0] < 0 || (!is_1q(g.kind) && loc[g.p1] < 0)) return false;
    t.r0 = reg[loc[g.p0]];
    t.r1 = is_1q(g.kind) ? 0 : reg[loc[g.p1]];
    if (t.r0 < 0 || t.r1 < 0 || (!is_1q(g.kind) && t.r0 == t.r1)) return false;
    if (g.kind == KROT) {
        t.kind = DK_ROT;
        t.r1 = g.p1;    // partial-sum slot
        t.cs = g.cs;    // axis
        for (int i = 0; i < 8; ++i) t.m[i] = R(g.m[i]);
        // the diagonal (d0, d1) again at m[8..11], for the axis-Z body
        t.m[8] = R(g.m[0]); t.m[9] = R(g.m[1]); t.m[10] = R(g.m[6]); t.m[11] = R(g.m[7]);
        return true;
    }
    const double* m = g.m;
    double m4[32];
    int kind = g.kind;
    if (kind == QSV_GC1Q && g.cs == 0) {
        // |0><0|_c (x) U + |1><1|_c (x) I on (c, t): a 4x4 in basis 2*x_c + x_t
        for (int i = 0; i < 32; ++i) m4[i] = 0.0;
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                m4[2 * (4 * r + c)] = m[2 * (2 * r + c)];
                m4[2 * (4 * r + c) + 1] = m[2 * (2 * r + c) + 1];
            }
        m4[2 * (4 * 2 + 2)] = 1.0;
        m4[2 * (4 * 3 + 3)] = 1.0;
        m = m4;
        kind = QSV_G2Q;
    }
    if (kind == QSV_G1Q) {
        if (is_zero(m[2]) && is_zero(m[3]) && is_zero(m[4]) && is_zero(m[5])) {
            t.kind = DK_1D;
            t.m[0] = R(m[0]); t.m[1] = R(m[1]); t.m[2] = R(m[6]); t.m[3] = R(m[7]);
        } else if (is_zero(m[1]) && is_zero(m[3]) && is_zero(m[5]) && is_zero(m[7])) {
            t.kind = DK_1R;
            for (int i = 0; i < 8; ++i) t.m[i] = R(m[i]);
        } else {
            t.kind = DK_1Q;
            for (int i = 0; i < 8; ++i) t.m[i] = R(m[i]);
        }
    } else if (kind == QSV_GC1Q) {
        const bool offzero = is_zero(m[2]) && is_zero(m[3]) && is_zero(m[4]) && is_zero(m[5]);
        const bool is_x = is_zero(m[0]) && is_zero(m[1]) && m[2] == 1.0 && is_zero(m[3]) &&
                          m[4] == 1.0 && is_zero(m[5]) && is_zero(m[6]) && is_zero(m[7]);
        if (is_x) {
            t.kind = DK_CX;
        } else if (offzero) {
            t.kind = DK_CD;
            t.m[0] = R(m[0]); t.m[1] = R(m[1]); t.m[2] = R(m[6]); t.m[3] = R(m[7]);
        } else {
            t.kind = DK_C1Q;
            for (int i = 0; i < 8; ++i) t.m[i] = R(m[i]);
        }
    } else {
        t.kind = DK_2Q;
        if (t.r0 < t.r1) {
            for (int i = 0; i < 32; ++i) t.m[i] = R(m[i]);
        } else {
            // exchange the two qubits: rows/columns permuted by (0, 2, 1, 3)
            static const int sg[4] = {0, 2, 1, 3};
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) {
                    t.m[2 * (4 * r + c)] = R(m[2 * (4 * sg[r] + sg[c])]);
                    t.m[2 * (4 * r + c) + 1] = R(m[2 * (4 * sg[r] + sg[c]) + 1]);
                }
            const int x = t.r0;
            t.r0 = t.r1;
            t.r1 = x;
        }
    }
    return true;
}

template <typename R, int K, int RB>
hipError_t launch_tile(qsv_ctx ctx, void* s, int n, bool split, const char* dplan, int from_zero) {
    using V = typename V2T<R>::type;
    const unsigned tiles = unsigned(uint64_t(1) << (n - K));
    if (split)
        hipLaunchKernelGGL((k_tile<R, K, RB, true>), dim3(tiles), dim3(1 << (K - RB)), 0, ctx->stream,
                           static_cast<V*>(s), dplan, from_zero);
    else
        hipLaunchKernelGGL((k_tile<R, K, RB, false>), dim3(tiles), dim3(1 << (K - RB)), 0, ctx->stream,
                           static_cast<V*>(s), dplan, from_zero);
    return hipGetLastError();
}

// The compiled (tile bits, register bits) shapes, 256 threads each.
template <typename R>
hipError_t launch_tile_k(qsv_ctx ctx, void* s, int n, int k, int rb, bool split, const char* dplan,
                         int fz) {
    switch (k * 8 + rb) {
    case 10 * 8 + 2: return launch_tile<R, 10, 2>(ctx, s, n, split, dplan, fz);
    case 11 * 8 + 3: return launch_tile<R, 11, 3>(ctx, s, n, split, dplan, fz);
    case 12 * 8 + 3: return launch_tile<R, 12, 3>(ctx, s, n, split, dplan, fz);
    case 12 * 8 + 4: return launch_tile<R, 12, 4>(ctx, s, n, split, dplan, fz);
    case 13 * 8 + 4: return launch_tile<R, 13, 4>(ctx, s, n, split, dplan, fz);
    case 13 * 8 + 5: return launch_tile<R, 13, 5>(ctx, s, n, split, dplan, fz);
    default: return hipErrorInvalidValue;
    }
}

// Bytes of a pass's device record (header, stages, gates; 256-byte
// aligned).  Fusion never adds gates, so the unfused count bounds the size.
template <typename R>
size_t record_bytes_t(const Pass& ps) {
    size_t b = sizeof(TPassHdr) + ps.stages.size() * sizeof(TStage) + ps.gates.size() * sizeof(TGate<R>);
    return (b + 255) & ~size_t(255);
}

// If the gate's matrix is a permutation matrix with unit entries (X, CX on
// either control state, SWAP), fill pi (if given) with the local-index map
// x -> row of the 1 in column x, and return true.  Local index: 1q -> the
// target bit; two positions -> 2*x_p0 + x_p1 (control = p0 for controlled).
bool permutation_of(const PGate& g, int* pi) {
    if (g.kind == KROT) return false;
    double m4[32];
    int d;
    if (g.kind == QSV_G1Q) {
        d = 2;
        for (int i = 0; i < 8; ++i) m4[i] = g.m[i];
    } else if (g.kind == QSV_GC1Q) {
        d = 4;
        for (int i = 0; i < 32; ++i) m4[i] = 0.0;
        const int c1 = g.cs & 1, c0 = 1 - c1;
        m4[2 * (4 * (2 * c0) + 2 * c0)] = 1.0;
        m4[2 * (4 * (2 * c0 + 1) + 2 * c0 + 1)] = 1.0;
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                m4[2 * (4 * (2 * c1 + r) + 2 * c1 + c)] = g.m[2 * (2 * r + c)];
                m4[2 * (4 * (2 * c1 + r) + 2 * c1 + c) + 1] = g.m[2 * (2 * r + c) + 1];
            }
    } else {
        d = 4;
        for (int i = 0; i < 32; ++i) m4[i] = g.m[i];
    }
    int p[4] = {-1, -1, -1, -1};
    for (int c = 0; c < d; ++c)
        for (int r = 0; r < d; ++r) {
            const double re = m4[2 * (d * r + c)], im = m4[2 * (d * r + c) + 1];
            if (im != 0.0) return false;
            if (re == 1.0) {
                if (p[c] >= 0) return false;
                p[c] = r;
            } else if (re != 0.0) {
                return false;
            }
        }
    for (int c = 0; c < d; ++c)
        if (p[c] < 0) return false;
    if (pi)
        for (int c = 0; c < d; ++c) pi[c] = p[c];
    return true;
}

// Thread-bit order of a stage: thread bit j <-> local tile bit tb[j], the
// complement of the stage's register bits.  Correctness does not depend on
// the order; LDS bank conflicts do.  An LDS access serves the lanes of a
// wave in groups, and the swizzle (tile_swz) sends local bit b of the
// (half-)tile index to bank field bit b mod F (F = 4 for 16-byte, 5 for
// 8-byte amplitudes).  So lanes 0..F-1 should take bits of distinct
// residues, the lower lanes the residues below F - 1 (groups of 8 lanes are
// then conflict-free as well as groups of 2^F), both for the reads into the
// stage (index without the bit hprev) and the writes out of it (without
// hnext).  Greedy, lane by lane; the first `fixed` lanes keep the ascending
// order (the coalesced runs of a global load or store), lanes from F on stay
// ascending.  Returns the number of thread bits.
int stage_thread_bits(const Stage& st, int k, int hprev, int hnext, int fixed, int elem_bytes,
                      int* tb) {
    const int F = elem_bytes == 16 ? 4 : 5;
    uint32_t used = 0;
    for (int j = 0; j < st.nr; ++j) used |= 1u << st.rbits[j];
    int cand[32], nc = 0;
    for (int b = 0; b < k; ++b)
        if (!((used >> b) & 1)) cand[nc++] = b;
    auto res = [F](int b, int h) { return (h >= 0 && b > h ? b - 1 : b) % F; };
    bool taken[32] = {};
    uint32_t seen_r = 0, seen_w = 0;
    for (int j = 0; j < nc; ++j) {
        int pick = -1;
        if (j < fixed || j >= F) {
            for (int c = 0; c < nc && pick < 0; ++c)
                if (!taken[c]) pick = c;
        } else {
            int best = -1;
            for (int c = 0; c < nc; ++c) {
                if (taken[c]) continue;
                const int rr = res(cand[c], hprev), rw = res(cand[c], hnext);
                const bool ok_r = !((seen_r >> rr) & 1) && (j == F - 1 || rr != F - 1);
                const bool ok_w = !((seen_w >> rw) & 1) && (j == F - 1 || rw != F - 1);
                const int score = int(ok_r) + int(ok_w);
                if (score > best) {
                    best = score;
                    pick = c;
                }
            }
        }
        taken[pick] = true;
        tb[j] = cand[pick];
        seen_r |= 1u << res(cand[pick], hprev);
        seen_w |= 1u << res(cand[pick], hnext);
    }
    return nc;
}

// Fill the device record of a tile pass at h.  False on a planner bug.
template <typename R>
bool write_record_t(char* h, const std::vector<PGate>& gates, const Pass& ps) {
    using V = typename V2T<R>::type;
    TPassHdr* hd = reinterpret_cast<TPassHdr*>(h);
    hd->k = ps.k;
    hd->nstages = int32_t(ps.stages.size());
    hd->pad = 0;
    int loc[64];
    for (int p = 0; p < 64; ++p) loc[p] = -1;
    for (int b = 0; b < 24; ++b) hd->pos[b] = b < ps.k ? ps.pos[b] : 0;
    for (int b = 0; b < ps.k; ++b) loc[ps.pos[b]] = b;
    const int rb = ps.rb;
    hd->rb = rb;
    hd->pad2 = 0;
    if (ps.stages.empty()) return false;
    const int ns = int(ps.stages.size());
    // Each stage's gates; trailing permutation gates (X, CX, SWAP: 0/1
    // matrices) whose bits no later gate of the stage touches are not run:
    // they only decide where each register slot is written at the stage's
    // end.  dest[si][u] = slot whose position slot u's amplitude takes.
    std::vector<std::vector<PGate>> run(static_cast<size_t>(ns));
    std::vector<std::array<int, 32>> dest(static_cast<size_t>(ns));
    for (int si = 0; si < ns; ++si) {
        const Stage& st = ps.stages[size_t(si)];
        int reg[32];
        for (int x = 0; x < 32; ++x) reg[x] = -1;
        for (int j = 0; j < st.nr; ++j) reg[st.rbits[j]] = j;
        std::vector<PGate> fused = fuse_stage(gates, st.gates);
        std::vector<char> virt(fused.size(), 0);
        uint32_t touched = 0;   // register bits used by later gates that run
        // split exchange: the bit shared with the next stage decides the write
        // round, so no permutation may move it
        const int hnext = (ps.split && si + 1 < ns) ? ps.stages[size_t(si) + 1].hprev : -1;
        if (hnext >= 0) {
            if (reg[hnext] < 0) return false;
            touched |= 1u << reg[hnext];
        }
        for (size_t i = fused.size(); i-- > 0;) {
            const PGate& fg = fused[i];
            const int b0 = loc[fg.p0] >= 0 ? reg[loc[fg.p0]] : -1;
            const int b1 = is_1q(fg.kind) ? b0 : (loc[fg.p1] >= 0 ? reg[loc[fg.p1]] : -1);
            if (b0 < 0 || b1 < 0) return false;
            const uint32_t bits = (1u << b0) | (1u << b1);
            if (!(bits & touched) && permutation_of(fg, nullptr)) virt[i] = 1;
            else touched |= bits;
        }
        std::array<int, 32>& D = dest[size_t(si)];
        for (int u = 0; u < 32; ++u) D[u] = u;
        for (size_t i = 0; i < fused.size(); ++i) {
            if (!virt[i]) {
                run[size_t(si)].push_back(fused[i]);
                continue;
            }
            // local index of the gate: 1q -> bit of p0; 2-position -> 2*x_p0 + x_p1
            const PGate& fg = fused[i];
            int pi[4];
            permutation_of(fg, pi);
            const int b0 = reg[loc[fg.p0]];
            const int b1 = is_1q(fg.kind) ? -1 : reg[loc[fg.p1]];
            for (int u = 0; u < (1 << rb); ++u) {
                const int x = D[u];
                const int li = b1 < 0 ? ((x >> b0) & 1) : (((x >> b0) & 1) << 1) | ((x >> b1) & 1);
                const int lo = pi[li];
                int y = x;
                if (b1 < 0) {
                    y = (y & ~(1 << b0)) | ((lo & 1) << b0);
                } else {
                    y = (y & ~((1 << b0) | (1 << b1))) | (((lo >> 1) & 1) << b0) | ((lo & 1) << b1);
                }
                D[u] = y;
            }
        }
    }
    // thread-bit order of every stage; the load mapping is the first
    // stage's, the store mapping the last stage's
    std::vector<std::array<int, 32>> tord(static_cast<size_t>(ns));
    for (int si = 0; si < ns; ++si) {
        const Stage& st = ps.stages[size_t(si)];
        const int hprev = ps.split ? st.hprev : -1;
        const int hnext = (ps.split && si + 1 < ns) ? ps.stages[size_t(si) + 1].hprev : -1;
        const int fixed = (si == 0 || si == ns - 1) ? ps.coal : 0;
        if (stage_thread_bits(st, ps.k, hprev, hnext, fixed, int(sizeof(V)), tord[size_t(si)].data()) !=
            ps.k - st.nr)
            return false;
    }
    auto mapping = [&](int si, const int* perm, int32_t* tpos, uint64_t* du) {
        const Stage& st = ps.stages[size_t(si)];
        const int nt = ps.k - st.nr;
        int tj = 0;
        for (; tj < nt && tj < 10; ++tj) tpos[tj] = ps.pos[tord[size_t(si)][size_t(tj)]];
        for (; tj < 10; ++tj) tpos[tj] = 0;
        for (int u = 0; u < 32; ++u) {
            uint64_t off = 0;
            if (u < (1 << rb)) {
                const int x = perm[u];
                for (int j = 0; j < rb; ++j)
                    if ((x >> j) & 1) off |= uint64_t(1) << ps.pos[st.rbits[j]];
            }
            du[u] = off;
        }
    };
    static const int ident[32] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15,
                                  16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31};
    mapping(0, ident, hd->tpos_ld, hd->du);
    mapping(ns - 1, dest[size_t(ns - 1)].data(), hd->tpos_st, hd->du_st);
    TStage* ts = reinterpret_cast<TStage*>(h + sizeof(TPassHdr));
    TGate<R>* tg = reinterpret_cast<TGate<R>*>(h + sizeof(TPassHdr) + ps.stages.size() * sizeof(TStage));
    int gi = 0;
    for (int si = 0; si < ns; ++si) {
        const Stage& st = ps.stages[size_t(si)];
        ts[si].gbeg = gi;
        int tj = 0;
        for (; tj < ps.k - st.nr && tj < 10; ++tj) ts[si].tbits[tj] = tord[size_t(si)][size_t(tj)];
        for (; tj < 10; ++tj) ts[si].tbits[tj] = 0;
        // split exchange: half-tile addresses without the shared bit
        const int hprev = ps.split ? st.hprev : -1;
        const int hnext = (ps.split && si + 1 < ns) ? ps.stages[size_t(si) + 1].hprev : -1;
        if (ps.split && si > 0 && (hprev < 0 || st.rbits[st.nr - 1] != hprev)) return false;
        auto drop = [](uint32_t e, int h) {   // remove local bit h from e
            return h < 0 ? e : ((e & ((1u << h) - 1)) | ((e >> (h + 1)) << h));
        };
        auto slot_off_h = [&](int u, int h) {
            uint32_t e = 0;
            for (int j = 0; j < st.nr; ++j)
                if ((u >> j) & 1) e |= 1u << st.rbits[j];
            return tile_swz(drop(e, h), int(sizeof(V))) * uint32_t(sizeof(V));
        };
        for (int u = 0; u < 32; ++u) {
            const bool in = u < (1 << st.nr);
            ts[si].su[u] = in ? slot_off_h(u, hprev) : 0;
            ts[si].su_wr[u] = in ? slot_off_h(dest[size_t(si)][u], hnext) : 0;
        }
        ts[si].jw = -1;
        if (hnext >= 0)
            for (int j = 0; j < st.nr; ++j)
                if (st.rbits[j] == hnext) ts[si].jw = j;
        if (hnext >= 0 && ts[si].jw < 0) return false;
        for (int j = 0; j < 10; ++j) {
            const int b = ts[si].tbits[j];
            ts[si].tbr[j] = (hprev >= 0 && b > hprev) ? b - 1 : b;
            ts[si].tbw[j] = (hnext >= 0 && b > hnext) ? b - 1 : b;
        }
        for (const PGate& fg : run[size_t(si)])
            if (!to_device_gate<R>(fg, loc, st, tg[gi++])) return false;
        ts[si].gend = gi;
    }
    hd->ngates = gi;
    return true;
}

template <typename R>
hipError_t run_passes_t(qsv_ctx ctx, void* s, int n, const std::vector<PGate>& gates,
                        const std::vector<Pass>& passes, bool cached, bool from_zero) {
    using V = typename V2T<R>::type;
    // upload layout: one record per tile pass
    size_t bytes = 0;
    std::vector<size_t> offs(passes.size(), 0);
    for (size_t i = 0; i < passes.size(); ++i) {
        if (passes[i].single) continue;
        if (passes[i].k < kMinTileBits || passes[i].k > TileK<R>::value ||
            n - passes[i].k > kMaxTileGridLog2)
            return hipErrorInvalidValue;
        offs[i] = bytes;
        bytes += record_bytes_t<R>(passes[i]);
    }
    char* dev = nullptr;
    const int dt0 = sizeof(R) == 8 ? QSV_C128 : QSV_C64;
    std::vector<hipFunction_t> jfns;   // specialised kernel of each pass (null: interpret)
    if (bytes && cached && ctx->plan_resident) {
        dev = static_cast<char*>(ctx->d_plan);
        if (ctx->jit_mode) jfns = ctx->jit_plan_fns;
    } else if (bytes) {
        void* host = nullptr;
        hipError_t e = plan_staging(ctx, bytes, &host);
        if (e != hipSuccess) return e;
        char* h = static_cast<char*>(host);
        for (size_t i = 0; i < passes.size(); ++i)
            if (!passes[i].single && !write_record_t<R>(h + offs[i], gates, passes[i]))
                return hipErrorInvalidValue;
        if (ctx->jit_mode) {
            std::vector<const char*> recs(passes.size(), nullptr);
            std::vector<bool> spl(passes.size(), false);
            for (size_t i = 0; i < passes.size(); ++i)
                if (!passes[i].single) {
                    recs[i] = h + offs[i];
                    spl[i] = passes[i].split;
                }
            e = jit_prepare(ctx, dt0, recs, spl, jfns);
            if (e != hipSuccess) return e;
            if (cached) ctx->jit_plan_fns = jfns;
        }
        void* d = nullptr;
        e = plan_upload(ctx, bytes, &d);
        if (e != hipSuccess) return e;
        dev = static_cast<char*>(d);
        ctx->plan_resident = cached;
    }
    const char* pname = sizeof(R) == 8 ? "tile_pass_c128" : "tile_pass_c64";
    const int dt = sizeof(R) == 8 ? QSV_C128 : QSV_C64;
    // from_zero: the first pass makes |0...0> itself when it is a tile pass;
    // otherwise the state is set first
    const bool gen_first = from_zero && !passes.empty() && !passes[0].single;
    if (from_zero && !gen_first) {
        hipError_t e = launch_init_basis(ctx, s, n, dt, 0);
        if (e != hipSuccess) return e;
    }
    for (size_t i = 0; i < passes.size(); ++i) {
        const Pass& ps = passes[i];
        hipError_t e;
        if (ps.single) {
            e = launch_gate(ctx, s, n, dt, gates[size_t(ps.gates[0])]);
        } else {
            const bool gen = gen_first && i == 0;   // writes the state without reading it
            prof_before(ctx, pname, (gen ? 1.0 : 2.0) * double(uint64_t(1) << n) * sizeof(V));
            if (i < jfns.size() && jfns[i]) {
                V* sv = static_cast<V*>(s);
                const char* pv = dev + offs[i];
                int fz = gen ? 1 : 0;
                void* args[] = {&sv, &pv, &fz};
                e = hipModuleLaunchKernel(jfns[i], unsigned(uint64_t(1) << (n - ps.k)), 1, 1,
                                          1u << (ps.k - ps.rb), 1, 1, 0, ctx->stream, args, nullptr);
            } else {
                e = launch_tile_k<R>(ctx, s, n, ps.k, ps.rb, ps.split, dev + offs[i], gen ? 1 : 0);
            }
            prof_after(ctx);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

size_t pass_record_bytes(int dtype, const Pass& ps) {
    return dtype == QSV_C128 ? record_bytes_t<double>(ps) : record_bytes_t<float>(ps);
}

bool write_pass_record(int dtype, char* dst, const std::vector<PGate>& gates, const Pass& ps) {
    return dtype == QSV_C128 ? write_record_t<double>(dst, gates, ps)
                             : write_record_t<float>(dst, gates, ps);
}

bool tile_shape_supported(int dtype, int tile_bits, int reg_bits) {
    (void)dtype;
    switch (tile_bits * 8 + reg_bits) {
    case 10 * 8 + 2: case 11 * 8 + 3: case 12 * 8 + 3: case 12 * 8 + 4: case 13 * 8 + 4:
    case 13 * 8 + 5: return true;
    default: return false;
    }
}

int tile_bits_max(int dtype) { return dtype == QSV_C128 ? TileK<double>::value : TileK<float>::value; }

hipError_t run_passes(qsv_ctx ctx, void* s, int n, int dtype, const std::vector<PGate>& gates,
                      const std::vector<Pass>& passes, bool cached, bool from_zero) {
    return dtype == QSV_C128 ? run_passes_t<double>(ctx, s, n, gates, passes, cached, from_zero)
                             : run_passes_t<float>(ctx, s, n, gates, passes, cached, from_zero);
}

}  // namespace qsv
