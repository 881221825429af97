// Fusion planner.
//
// Passes: a pass covers a set S of index-bit positions (|S| = tile bits,
// always containing the lowest `low_bits` positions so every tile is made of
// contiguous runs); every gate of the pass acts only on positions in S, so
// one HBM read and one HBM write of the state apply the whole group.  Gates
// are scanned in circuit order.  A gate joins the current pass if its
// positions fit in S (growing S while room is left) and none of its
// positions is "blocked"; a gate that cannot join is deferred and blocks its
// positions for the rest of the scan, so no later gate on those qubits can
// overtake it.  Gates that join therefore only overtake deferred gates on
// disjoint qubits, with which they commute.
//
// Stages: inside a tile of 2^k amplitudes each of the 256 threads holds
// 2^(k-8) amplitudes in registers, spanning k-8 "register bits" of the
// tile; a gate is applied in registers when all its bits are register bits.
// Stage 0 uses the load mapping (register bits = the k-8 highest local
// bits, thread bits = the 8 lowest, which keeps global accesses
// coalesced); later stages re-map through LDS; the last stage again uses
// the load mapping so the store is coalesced.  The same blocking rule
// orders gates across stages, and a stage's register bits are chosen the way
// a pass's bits are (the addition that lets the stage take the most gates).
#include <algorithm>
#include <complex>
#include <cstring>

#include "qsv_internal.h"

namespace qsv {

// A gate with extra controls is a barrier: its mask covers every position
// plus bit 63, which no tile set ever holds (positions are < 36), so no
// pass can take it, even one whose tile spans the whole state, and no later
// gate can overtake it; the planner gives it a pass of its own when it
// reaches the front.
constexpr uint64_t kBarrierBit = uint64_t(1) << 63;
static inline uint64_t gate_mask(const PGate& g, int n) {
    if (g.cm) return ((uint64_t(1) << n) - 1) | kBarrierBit;
    uint64_t m = uint64_t(1) << g.p0;
    if (!is_1q(g.kind)) m |= uint64_t(1) << g.p1;
    return m;
}

// Greedy scan: take gates of `rem` whose bits fit in S (|S| <= cap, S may
// grow unless `fixed`); the rest are deferred with their bits blocked.
static void greedy(const std::vector<int>& rem, const std::vector<uint64_t>& masks, uint64_t& S,
                   int cap, bool fixed, std::vector<int>& take, std::vector<int>& defer) {
    uint64_t blocked = 0;
    int cnt = __builtin_popcountll(S);
    for (int gi : rem) {
        const uint64_t gm = masks[size_t(gi)];
        if (gm & blocked) {
            defer.push_back(gi);
            blocked |= gm;
            continue;
        }
        const uint64_t need = gm & ~S;
        const int add = __builtin_popcountll(need);
        if (add == 0 || (!fixed && cnt + add <= cap)) {
            S |= need;
            cnt += add;
            take.push_back(gi);
        } else {
            defer.push_back(gi);
            blocked |= gm;
        }
    }
}

// Number of gates of `rem` (circuit order) that a pass over the fixed bit
// set S takes under the blocking rule; the scan stops once every bit of S is
// blocked, since no later gate can join then.
static size_t closure_count(const std::vector<int>& rem, size_t lim, const std::vector<uint64_t>& masks,
                            uint64_t S) {
    uint64_t blocked = 0;
    size_t cnt = 0;
    for (size_t j = 0; j < lim; ++j) {
        const uint64_t gm = masks[size_t(rem[j])];
        if (!(gm & ~S) && !(gm & blocked)) {
            ++cnt;
        } else {
            blocked |= gm;
            if ((blocked & S) == S) break;
        }
    }
    return cnt;
}

// Bit set of the next pass: start from the low bits and repeatedly add the
// bits of one not-yet-blocked gate, choosing the addition after which the
// pass takes the most gates (ties: fewer new bits, then circuit order),
// until no gate's bits fit in the K positions.  This looks past the first
// gates in circuit order, which an in-order greedy fill would commit to.
// remaining gate count below which the planner searches the tail; a second
// plan that searches from further back (kTailLookGatesWide) is kept only if
// it needs fewer passes (a plan of the same count can run slower, since its
// passes carry different gates)
constexpr size_t kTailLookGates = 400;
constexpr size_t kTailLookGatesWide = 1000;

static uint64_t choose_bits(const std::vector<int>& rem, const std::vector<uint64_t>& masks, uint64_t S, int K) {
    const size_t lim = std::min(rem.size(), size_t(4096));
    for (;;) {
        const int have = __builtin_popcountll(S);
        if (have >= K) break;
        uint64_t cand[64];
        int nc = 0;
        uint64_t blocked = 0;
        for (size_t j = 0; j < lim && nc < 64; ++j) {
            const uint64_t gm = masks[size_t(rem[j])];
            const uint64_t need = gm & ~S;
            if (need && !(gm & blocked) && have + __builtin_popcountll(need) <= K) {
                bool dup = false;
                for (int c = 0; c < nc; ++c) dup |= cand[c] == need;
                if (!dup) cand[nc++] = need;
            }
            if (need || (gm & blocked)) blocked |= gm;
            if (__builtin_popcountll(blocked & ~S) + have >= 64) break;
        }
        if (nc == 0) break;
        size_t best_cnt = 0;
        int best = -1;
        for (int c = 0; c < nc; ++c) {
            const size_t cnt = closure_count(rem, lim, masks, S | cand[c]);
            if (best < 0 || cnt > best_cnt ||
                (cnt == best_cnt && __builtin_popcountll(cand[c]) < __builtin_popcountll(cand[best]))) {
                best = c;
                best_cnt = cnt;
            }
        }
        S |= cand[best];
    }
    return S;
}

static void plan_stages(int n, const std::vector<PGate>& gates, Pass& ps) {
    (void)n;
    const int K = ps.k;
    const int RB = ps.rb;
    const int C = std::min(ps.coal, K - RB);
    const bool split = ps.split;
    int loc[64];
    for (int p = 0; p < 64; ++p) loc[p] = -1;
    for (int b = 0; b < K; ++b) loc[ps.pos[b]] = b;
    // gate masks in local-bit coordinates, indexed by global gate index
    std::vector<uint64_t> lm(gates.size(), 0);
    for (int gi : ps.gates) {
        const PGate& g = gates[size_t(gi)];
        uint64_t m = uint64_t(1) << loc[g.p0];
        if (!is_1q(g.kind)) m |= uint64_t(1) << loc[g.p1];
        lm[size_t(gi)] = m;
    }
    const uint64_t lanes = (uint64_t(1) << C) - 1;   // bits the first/last stage keep on lanes
    auto mask_of = [&](const Stage& st) {
        uint64_t m = 0;
        for (int j = 0; j < st.nr; ++j) m |= uint64_t(1) << st.rbits[j];
        return m;
    };
    // A register set of RB bits containing S; padding prefers the highest
    // free bits, and never the lane bits when `avoid` is set.  With a split
    // exchange the set shares a bit h with `prev` (the previous stage's
    // set), which goes last in the register order.
    auto make_stage = [&](uint64_t S, bool avoid, uint64_t prev, std::vector<int>&& g) {
        Stage st;
        st.nr = RB;
        int h = -1;
        if (split && prev) {
            const uint64_t common = S & prev;
            const uint64_t cand = common ? common : (prev & ~(avoid ? lanes : 0));
            if (cand) h = 63 - __builtin_clzll(cand);   // highest candidate
            if (h >= 0) S |= uint64_t(1) << h;
        }
        for (int b = K - 1; b >= 0 && __builtin_popcountll(S) < RB; --b)
            if (!((S >> b) & 1) && !(avoid && ((lanes >> b) & 1))) S |= uint64_t(1) << b;
        int j = 0;
        for (int b = 0; b < K && j < RB; ++b)
            if (((S >> b) & 1) && b != h) st.rbits[j++] = b;
        if (h >= 0) st.rbits[j++] = h;
        st.hprev = h;
        st.gates = std::move(g);
        return st;
    };
    // greedy scan that may not use the lane bits (first stage)
    auto greedy_avoid = [&](const std::vector<int>& rem, uint64_t& S, std::vector<int>& take,
                            std::vector<int>& defer) {
        uint64_t blocked = 0;
        for (int gi : rem) {
            const uint64_t gm = lm[size_t(gi)];
            if ((gm & blocked) || (gm & lanes)) {
                defer.push_back(gi);
                blocked |= gm;
                continue;
            }
            const uint64_t need = gm & ~S;
            if (__builtin_popcountll(S | need) <= RB) {
                S |= need;
                take.push_back(gi);
            } else {
                defer.push_back(gi);
                blocked |= gm;
            }
        }
    };

    // The bits of each stage are chosen the way a pass chooses its bits
    // (choose_bits: the addition after which the stage takes the most gates),
    // not by an in-order fill, which commits to the first gates' bits and
    // leaves more stages -- and LDS exchanges -- per pass.  For the first
    // stage, gates on lane bits get bits no register set can hold.
    constexpr uint64_t kNoFit = ~uint64_t(0) << 48;   // 16 bits above every local bit
    std::vector<uint64_t> lm0(lm);
    for (int gi : ps.gates)
        if (lm[size_t(gi)] & lanes) lm0[size_t(gi)] |= kNoFit;
    ps.stages.clear();
    std::vector<int> rem = ps.gates, take, defer;
    uint64_t S = choose_bits(rem, lm0, 0, RB);
    greedy_avoid(rem, S, take, defer);
    ps.stages.push_back(make_stage(S, true, 0, std::move(take)));
    rem.swap(defer);
    while (!rem.empty()) {
        const uint64_t prev = mask_of(ps.stages.back());
        take.clear();
        defer.clear();
        S = choose_bits(rem, lm, 0, RB);
        greedy(rem, lm, S, RB, false, take, defer);
        if (split && !(S & prev) && __builtin_popcountll(S) == RB) {
            // a bit shared with the previous stage is needed: leave room for
            // one, or start the search from one of the previous stage's bits
            // (then gates on it join for free), whichever takes more gates
            take.clear();
            defer.clear();
            S = choose_bits(rem, lm, 0, RB - 1);
            greedy(rem, lm, S, RB - 1, false, take, defer);
            std::vector<int> t2, d2;
            for (uint64_t pb = prev; pb; pb &= pb - 1) {
                uint64_t S2 = choose_bits(rem, lm, pb & (~pb + 1), RB);
                t2.clear();
                d2.clear();
                greedy(rem, lm, S2, RB, false, t2, d2);
                if (t2.size() > take.size()) {
                    S = S2;
                    take.swap(t2);
                    defer.swap(d2);
                }
            }
        }
        uint64_t used = 0;
        for (int gi : take) used |= lm[size_t(gi)];
        // a stage that avoids the lane bits can also be the store stage
        bool avoid = (used & lanes) == 0;
        if (avoid && split && !(S & prev) && !(prev & ~lanes)) avoid = false;   // shared bit is a lane bit
        ps.stages.push_back(make_stage(S, avoid, prev, std::move(take)));
        rem.swap(defer);
    }
    // The store needs a stage that keeps the lane bits on lanes.  If the last
    // stage uses them, try to re-split the gates of the last two stages so
    // that the gates on lane bits all run in the first of the two and the
    // second avoids the lanes: that saves the empty store stage (one LDS
    // exchange).  The gates keep their order and the blocking rule, as in
    // every stage.
    const size_t ns = ps.stages.size();
    if (ns >= 3 && (mask_of(ps.stages.back()) & lanes)) {
        std::vector<int> G = ps.stages[ns - 2].gates;
        G.insert(G.end(), ps.stages[ns - 1].gates.begin(), ps.stages[ns - 1].gates.end());
        const uint64_t prevA = mask_of(ps.stages[ns - 3]);
        uint64_t seed = 0;
        for (int gi : G)
            if (lm[size_t(gi)] & lanes) seed |= lm[size_t(gi)];
        if (__builtin_popcountll(seed) <= RB) {
            uint64_t SA = choose_bits(G, lm, seed, RB);
            std::vector<int> ta, da;
            greedy(G, lm, SA, RB, false, ta, da);
            bool ok = (SA & seed) == seed && !(split && !(SA & prevA) && __builtin_popcountll(SA) == RB);
            uint64_t SB = 0;
            for (int gi : da) {
                ok &= !(lm[size_t(gi)] & lanes);
                SB |= lm[size_t(gi)];
            }
            ok &= __builtin_popcountll(SB) <= RB;
            if (ok) {
                uint64_t usedA = 0;
                for (int gi : ta) usedA |= lm[size_t(gi)];
                Stage A = make_stage(SA, (usedA & lanes) == 0, prevA, std::move(ta));
                const uint64_t mA = mask_of(A);
                // B shares a bit with A that is off the lanes (B holds no lane bit)
                ok = !(split && ((!(SB & mA) && __builtin_popcountll(SB) == RB) || !(mA & ~lanes)));
                if (ok) {
                    Stage B = make_stage(SB, true, mA, std::move(da));
                    if (!(mask_of(B) & lanes)) {
                        ps.stages[ns - 2] = std::move(A);
                        ps.stages[ns - 1] = std::move(B);
                    }
                }
            }
        }
    }
    if (mask_of(ps.stages.back()) & lanes) {
        uint64_t prev = mask_of(ps.stages.back());
        if (split && !(prev & ~lanes)) {
            // no bit to share that is off the lanes: an empty stage in between
            ps.stages.push_back(make_stage(0, false, prev, {}));
            prev = mask_of(ps.stages.back());
        }
        ps.stages.push_back(make_stage(0, true, prev, {}));
    }
}

// ------------------------------------------------------------ stage fusion
namespace {

using cd = std::complex<double>;

struct M4 { cd a[16]; };   // 4x4 row-major, basis 2*x_hi + x_lo of (qa, qb)

M4 m4_from(const double* m) {
    M4 r;
    for (int i = 0; i < 16; ++i) r.a[i] = cd(m[2 * i], m[2 * i + 1]);
    return r;
}
void m4_to(const M4& x, double* m) {
    for (int i = 0; i < 16; ++i) {
        m[2 * i] = x.a[i].real();
        m[2 * i + 1] = x.a[i].imag();
    }
}
M4 mul(const M4& x, const M4& y) {
    M4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cd acc = 0;
            for (int k = 0; k < 4; ++k) acc += x.a[4 * i + k] * y.a[4 * k + j];
            r.a[4 * i + j] = acc;
        }
    return r;
}
// A (x) B for 2x2 A (first qubit) and B (second)
M4 kron(const cd* A, const cd* B) {
    M4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r.a[4 * i + j] = A[2 * (i >> 1) + (j >> 1)] * B[2 * (i & 1) + (j & 1)];
    return r;
}
// exchange the roles of the two qubits: permute rows/columns by (0, 2, 1, 3)
M4 swapq(const M4& x) {
    static const int sg[4] = {0, 2, 1, 3};
    M4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r.a[4 * i + j] = x.a[4 * sg[i] + sg[j]];
    return r;
}
void m2_from(const double* m, cd* u) {
    for (int i = 0; i < 4; ++i) u[i] = cd(m[2 * i], m[2 * i + 1]);
}
void m2_mul(const cd* x, const cd* y, cd* r) {   // r = x y
    cd t[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) t[2 * i + j] = x[2 * i] * y[j] + x[2 * i + 1] * y[2 + j];
    for (int i = 0; i < 4; ++i) r[i] = t[i];
}

// the 4x4 of a 2-position gate in the basis 2*x_p0 + x_p1
M4 as4(const PGate& g) {
    if (g.kind == QSV_G2Q) return m4_from(g.m);
    // controlled: |~cs><~cs| (x) I + |cs><cs| (x) U on (control = p0, target = p1)
    M4 r;
    for (int i = 0; i < 16; ++i) r.a[i] = 0;
    cd u[4];
    m2_from(g.m, u);
    const int c1 = g.cs, c0 = 1 - g.cs;
    r.a[4 * (2 * c0) + 2 * c0] = 1;
    r.a[4 * (2 * c0 + 1) + 2 * c0 + 1] = 1;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) r.a[4 * (2 * c1 + i) + 2 * c1 + j] = u[2 * i + j];
    return r;
}

}  // namespace

// Arithmetic cost of a gate in real FMAs per amplitude, as the tile kernel
// applies it: dense 1q 8, diagonal 1q 4, controlled 1q 4 (half the
// amplitudes), controlled X 0 (a register swap), controlled diagonal 2,
// dense 2q 16 (a control on state 0 is applied as a dense 2q).
static bool offdiag_zero(const double* m) { return m[2] == 0.0 && m[3] == 0.0 && m[4] == 0.0 && m[5] == 0.0; }
static bool is_pauli_x(const double* m) {
    return m[0] == 0.0 && m[1] == 0.0 && m[2] == 1.0 && m[3] == 0.0 && m[4] == 1.0 && m[5] == 0.0 &&
           m[6] == 0.0 && m[7] == 0.0;
}
static int gate_cost(const PGate& g) {
    switch (g.kind) {
    case QSV_G1Q: return offdiag_zero(g.m) ? 4 : 8;
    case QSV_GC1Q:
        if (g.cs == 0) return 16;
        return is_pauli_x(g.m) ? 0 : offdiag_zero(g.m) ? 2 : 4;
    case KROT: return 8;
    default: return 16;
    }
}
static int cost1(const cd* u) { return (u[1] == 0.0 && u[2] == 0.0) ? 4 : 8; }

std::vector<PGate> fuse_stage(const std::vector<PGate>& gates, const std::vector<int>& idx) {
    std::vector<PGate> out;
    out.reserve(idx.size());   // fusion never adds gates
    bool has[64] = {false};
    cd pend[64][4];
    // index in `out` of the last emitted gate touching each position (-1: none)
    int last[64];
    for (int p = 0; p < 64; ++p) last[p] = -1;

    // emit the pending 1-qubit product on position p: folded into the last
    // gate on p when that costs nothing (a 1q gate on p, or a dense 2q gate;
    // no gate on p follows it, so left-multiplying it is exact), else as a
    // gate of its own
    auto flush = [&](int p) {
        if (!has[p]) return;
        has[p] = false;
        const int l = last[p];
        if (l >= 0 && out[size_t(l)].kind == QSV_G1Q && !out[size_t(l)].cm) {
            PGate& o = out[size_t(l)];
            cd u[4];
            m2_from(o.m, u);
            m2_mul(pend[p], u, u);
            for (int i = 0; i < 4; ++i) {
                o.m[2 * i] = u[i].real();
                o.m[2 * i + 1] = u[i].imag();
            }
            return;
        }
        if (l >= 0 && out[size_t(l)].kind == QSV_G2Q && !out[size_t(l)].cm) {
            PGate& o = out[size_t(l)];
            static const cd I2[4] = {1, 0, 0, 1};
            const M4 L = o.p0 == p ? kron(pend[p], I2) : kron(I2, pend[p]);
            m4_to(mul(L, m4_from(o.m)), o.m);
            return;
        }
        PGate f{};
        f.kind = QSV_G1Q;
        f.p0 = p;
        f.cs = 1;
        for (int i = 0; i < 4; ++i) {
            f.m[2 * i] = pend[p][i].real();
            f.m[2 * i + 1] = pend[p][i].imag();
        }
        out.push_back(f);
        last[p] = int(out.size()) - 1;
    };

    for (int gi : idx) {
        const PGate& g = gates[size_t(gi)];
        if (g.cm) {
            // extra controls: pending products on its qubits and controls go
            // first, the gate stays whole, and nothing folds into it later
            uint64_t own = g.cm | (uint64_t(1) << g.p0);
            if (!is_1q(g.kind)) own |= uint64_t(1) << g.p1;
            for (int p = 0; p < 64; ++p)
                if ((own >> p) & 1) flush(p);
            out.push_back(g);
            for (int p = 0; p < 64; ++p)
                if ((own >> p) & 1) last[p] = int(out.size()) - 1;
            continue;
        }
        if (g.kind == KROT) {
            // kept whole (its partial sum is taken at this point)
            flush(g.p0);
            out.push_back(g);
            last[g.p0] = int(out.size()) - 1;
            continue;
        }
        if (g.kind == QSV_G1Q) {
            cd u[4];
            m2_from(g.m, u);
            if (has[g.p0]) m2_mul(u, pend[g.p0], pend[g.p0]);
            else {
                for (int i = 0; i < 4; ++i) pend[g.p0][i] = u[i];
                has[g.p0] = true;
            }
            continue;
        }
        const int a = g.p0, b = g.p1;
        // the previous gate, if it is the last one on both positions and acts
        // on exactly this pair (pending 1q gates on a, b lie between the two)
        int prev = -1;
        if (last[a] >= 0 && last[a] == last[b]) {
            const PGate& o = out[size_t(last[a])];
            if (!is_1q(o.kind) && o.kind != KROT && !o.cm &&
                ((o.p0 == a && o.p1 == b) || (o.p0 == b && o.p1 == a)))
                prev = last[a];
        }
        // fuse into one dense 2q gate only where that does not add arithmetic
        const int pend_cost = (has[a] ? cost1(pend[a]) : 0) + (has[b] ? cost1(pend[b]) : 0);
        const int own = gate_cost(g) + pend_cost;
        bool merge_prev = prev >= 0 && 16 <= own + gate_cost(out[size_t(prev)]);
        const bool absorb = (has[a] || has[b]) && (merge_prev || 16 <= own);
        if (!absorb && !merge_prev) {
            flush(a);
            flush(b);
            out.push_back(g);
            last[a] = last[b] = int(out.size()) - 1;
            continue;
        }
        M4 M = as4(g);   // basis (a, b)
        if (absorb) {
            static const cd I2[4] = {1, 0, 0, 1};
            const cd* ua = has[a] ? pend[a] : I2;
            const cd* ub = has[b] ? pend[b] : I2;
            M = mul(M, kron(ua, ub));
            has[a] = has[b] = false;
        }
        if (merge_prev) {
            PGate& o = out[size_t(prev)];
            M4 P = as4(o);
            if (o.p0 != a) P = swapq(P);   // express the earlier gate in basis (a, b)
            M = mul(M, P);
            o.kind = QSV_G2Q;
            o.p0 = a;
            o.p1 = b;
            o.cs = 1;
            m4_to(M, o.m);
        } else {
            PGate f{};
            f.kind = QSV_G2Q;
            f.p0 = a;
            f.p1 = b;
            f.cs = 1;
            m4_to(M, f.m);
            out.push_back(f);
            last[a] = last[b] = int(out.size()) - 1;
        }
    }
    for (int p = 0; p < 64; ++p) flush(p);
    return out;
}

// A square root of a 2x2 unitary U that is itself unitary: for a 2x2
// matrix, R = (U + s I) / t with s^2 = det U and t^2 = tr U + 2 s squares
// to U (Cayley-Hamilton); R is a polynomial in U, so it is normal with
// unit-modulus eigenvalues, i.e. unitary.  The sign of s is chosen so that
// t is not zero.
void unitary_sqrt2(const double* u, double* r) {
    const cd a(u[0], u[1]), b(u[2], u[3]), c(u[4], u[5]), d(u[6], u[7]);
    cd s = std::sqrt(a * d - b * c);
    cd t = std::sqrt(a + d + 2.0 * s);
    if (std::abs(t) < 1e-8) {
        s = -s;
        t = std::sqrt(a + d + 2.0 * s);
    }
    const cd m[4] = {(a + s) / t, b / t, c / t, (d + s) / t};
    for (int i = 0; i < 4; ++i) {
        r[2 * i] = m[i].real();
        r[2 * i + 1] = m[i].imag();
    }
}

// A 1-qubit gate with exactly two controls (a Toffoli, a doubly-controlled
// U; Sec. 2.4) becomes the exact two-qubit sequence of Barenco et al. 1995
// (Lemma 6.1), with V^2 = U:
//     C_c2(V)_t, CX(c1 -> c2), C_c2(V^dagger)_t, CX(c1 -> c2), C_c1(V)_t
// (controls on state 0 are wrapped in X on that control).  Its gates then
// fuse into tile passes like any other; gates with more controls, or with a
// 2-qubit base, stay barriers that run as passes of their own.
std::vector<PGate> expand_double_controls(const std::vector<PGate>& gates) {
    std::vector<PGate> out;
    out.reserve(gates.size());
    for (const PGate& g : gates) {
        int c[2], v[2], nc = 0, t = -1;
        bool ok = g.cm != 0 && (g.kind == QSV_G1Q || g.kind == QSV_GC1Q);
        if (ok) {
            if (g.kind == QSV_GC1Q) {
                c[nc] = g.p0;
                v[nc++] = g.cs;
                t = g.p1;
            } else {
                t = g.p0;
            }
            for (int p = 0; p < 64 && ok; ++p)
                if ((g.cm >> p) & 1) {
                    if (nc == 2) ok = false;
                    else {
                        c[nc] = p;
                        v[nc++] = int((g.cv >> p) & 1);
                    }
                }
            ok = ok && nc == 2;
        }
        if (!ok) {
            out.push_back(g);
            continue;
        }
        static const double X[8] = {0, 0, 1, 0, 1, 0, 0, 0};
        auto one = [&](int p, const double* m) {
            PGate x{};
            x.kind = QSV_G1Q;
            x.p0 = p;
            x.cs = 1;
            std::memcpy(x.m, m, 8 * sizeof(double));
            out.push_back(x);
        };
        auto ctl = [&](int pc, int pt, const double* m) {
            PGate x{};
            x.kind = QSV_GC1Q;
            x.p0 = pc;
            x.p1 = pt;
            x.cs = 1;
            std::memcpy(x.m, m, 8 * sizeof(double));
            out.push_back(x);
        };
        double vm[8], vd[8];
        unitary_sqrt2(g.m, vm);
        for (int r = 0; r < 2; ++r)
            for (int k = 0; k < 2; ++k) {
                vd[2 * (2 * r + k)] = vm[2 * (2 * k + r)];
                vd[2 * (2 * r + k) + 1] = -vm[2 * (2 * k + r) + 1];
            }
        for (int i = 0; i < 2; ++i)
            if (!v[i]) one(c[i], X);
        ctl(c[1], t, vm);
        ctl(c[0], c[1], X);
        ctl(c[1], t, vd);
        ctl(c[0], c[1], X);
        ctl(c[0], t, vm);
        for (int i = 0; i < 2; ++i)
            if (!v[i]) one(c[i], X);
    }
    return out;
}

std::vector<PGate> prefuse(const std::vector<PGate>& gates) {
    bool any_cm = false;
    for (const PGate& g : gates) any_cm |= g.cm != 0;
    std::vector<PGate> ex;
    if (any_cm) ex = expand_double_controls(gates);
    const std::vector<PGate>& src = any_cm ? ex : gates;
    std::vector<int> all(src.size());
    for (size_t i = 0; i < src.size(); ++i) all[i] = int(i);
    return fuse_stage(src, all);
}

void plan_pass_stages(int n, const std::vector<PGate>& gates, Pass& ps) { plan_stages(n, gates, ps); }

// Passes the greedy planner needs for `rem` (bit sets only, no stages).
static int count_passes(std::vector<int> rem, const std::vector<uint64_t>& masks, uint64_t low, int K) {
    int np = 0;
    std::vector<int> take, defer;
    while (!rem.empty()) {
        uint64_t S = choose_bits(rem, masks, low, K);
        take.clear();
        defer.clear();
        greedy(rem, masks, S, K, true, take, defer);
        if (take.empty()) {   // a barrier gate at the front: a pass of its own
            defer.erase(defer.begin());
        }
        rem.swap(defer);
        ++np;
    }
    return np;
}

// Near the end of a circuit the pass-by-pass choice can leave a last pass
// of a few gates that still costs a full read and write of the state.  When
// few gates remain, try as this pass's bit set the completion of every
// first gate choice (not only the best-scoring one) and keep the set after
// which the fewest passes remain; ties keep the default choice.
static uint64_t choose_bits_tail(const std::vector<int>& rem, const std::vector<uint64_t>& masks, uint64_t low,
                                 int K, uint64_t S_def) {
    auto passes_after = [&](uint64_t S) {
        std::vector<int> take, defer;
        greedy(rem, masks, S, K, true, take, defer);
        return take.empty() ? 1 << 30 : 1 + count_passes(std::move(defer), masks, low, K);
    };
    int best_np = passes_after(S_def);
    if (best_np <= 1) return S_def;
    uint64_t best = S_def;
    uint64_t tried[64];
    int nt = 0;
    uint64_t blocked = 0;
    const int have = __builtin_popcountll(low);
    for (size_t j = 0; j < rem.size() && nt < 64; ++j) {
        const uint64_t gm = masks[size_t(rem[j])];
        const uint64_t need = gm & ~low;
        if (need && !(gm & blocked) && have + __builtin_popcountll(need) <= K) {
            bool dup = false;
            for (int c = 0; c < nt; ++c) dup |= tried[c] == need;
            if (!dup) {
                tried[nt++] = need;
                const uint64_t S = choose_bits(rem, masks, low | need, K);
                if (S != best) {
                    const int np = passes_after(S);
                    if (np < best_np) {
                        best_np = np;
                        best = S;
                    }
                }
            }
        }
        if (need || (gm & blocked)) blocked |= gm;
    }
    return best;
}

static std::vector<Pass> plan_passes_tail(int n, const std::vector<PGate>& gates, const TileConfig& cfg,
                                          size_t tail_gates) {
    std::vector<Pass> passes;
    std::vector<uint64_t> masks(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) masks[i] = gate_mask(gates[i], n);
    if (n < kMinTileBits || cfg.tile_bits < kMinTileBits) {
        for (size_t i = 0; i < gates.size(); ++i) {
            Pass ps;
            ps.single = true;
            ps.k = 0;
            ps.gates.push_back(int(i));
            passes.push_back(std::move(ps));
        }
        return passes;
    }
    // a launch covers at most 2^32 - 1 work-items: 2^(n - K) tiles of 256
    // threads need n - K <= 23, so very large states take larger tiles
    const int K = std::max(std::min(cfg.tile_bits, n), std::min(n - kMaxTileGridLog2, kMaxTileBits));
    const int L = std::min(cfg.low_bits, K);
    std::vector<int> rem(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) rem[i] = int(i);

    while (!rem.empty()) {
        if (gates[size_t(rem[0])].cm) {
            Pass ps;
            ps.single = true;
            ps.k = K;
            ps.gates.push_back(rem[0]);
            passes.push_back(std::move(ps));
            rem.erase(rem.begin());
            continue;
        }
        const uint64_t low = (uint64_t(1) << L) - 1;
        uint64_t S = choose_bits(rem, masks, low, K);
        if (rem.size() <= tail_gates) S = choose_bits_tail(rem, masks, low, K, S);
        std::vector<int> take, defer;
        take.reserve(rem.size());
        greedy(rem, masks, S, K, true, take, defer);
        int cnt = __builtin_popcountll(S);
        // fill the tile up to K positions with the lowest unused ones
        for (int p = 0; p < n && cnt < K; ++p) {
            if (!((S >> p) & 1)) {
                S |= uint64_t(1) << p;
                ++cnt;
            }
        }
        Pass ps;
        ps.single = (take.size() == 1);
        ps.k = K;
        ps.rb = tile_shape_supported(QSV_C128, K, cfg.reg_bits) ? cfg.reg_bits : K - 8;
        ps.coal = cfg.coal_bits;
        // a shared register bit leaves RB - 1 >= 2 bits for a 2-qubit gate
        ps.split = cfg.split != 0 && ps.rb >= 3;
        int i = 0;
        for (int p = 0; p < n; ++p)
            if ((S >> p) & 1) ps.pos[i++] = p;
        ps.gates = std::move(take);
        if (!ps.single) plan_stages(n, gates, ps);
        passes.push_back(std::move(ps));
        rem.swap(defer);
    }
    return passes;
}

std::vector<Pass> plan_passes(int n, const std::vector<PGate>& gates, const TileConfig& cfg) {
    std::vector<Pass> passes = plan_passes_tail(n, gates, cfg, kTailLookGates);
    if (gates.size() > kTailLookGates && passes.size() > 2) {
        std::vector<Pass> wide = plan_passes_tail(n, gates, cfg, kTailLookGatesWide);
        if (wide.size() < passes.size()) passes = std::move(wide);
    }
    return passes;
}

const std::vector<Pass>& plan_memo(PlanMemo& m, int n, const std::vector<PGate>& fused, const TileConfig& cfg) {
    std::vector<uint32_t> sig(fused.size());
    for (size_t i = 0; i < fused.size(); ++i) {
        const PGate& g = fused[i];
        sig[i] = uint32_t(g.kind & 31) | (uint32_t(g.p0 & 63) << 5) |
                 (uint32_t(is_1q(g.kind) ? 0 : (g.p1 & 63)) << 11) | (uint32_t(g.cs & 1) << 17) |
                 (uint32_t(g.cm != 0) << 18);
    }
    const bool same = m.n == n && m.cfg.tile_bits == cfg.tile_bits && m.cfg.low_bits == cfg.low_bits &&
                      m.cfg.reg_bits == cfg.reg_bits && m.cfg.coal_bits == cfg.coal_bits &&
                      m.cfg.split == cfg.split && m.sig == sig;
    if (!same) {
        m.passes = plan_passes(n, fused, cfg);
        m.n = n;
        m.cfg = cfg;
        m.sig = std::move(sig);
    }
    return m.passes;
}

}  // namespace qsv
