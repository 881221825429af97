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
// the load mapping so the store is coalesced.  The same greedy, blocking
// rule orders gates across stages.
#include <algorithm>

#include "qsv_internal.h"

namespace qsv {

static inline uint64_t gate_mask(const PGate& g) {
    uint64_t m = uint64_t(1) << g.p0;
    if (g.kind != QSV_G1Q) m |= uint64_t(1) << g.p1;
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

static void plan_stages(int n, const std::vector<PGate>& gates, Pass& ps) {
    (void)n;
    const int K = ps.k;
    const int RB = K - 8;
    int loc[64];
    for (int p = 0; p < 64; ++p) loc[p] = -1;
    for (int b = 0; b < K; ++b) loc[ps.pos[b]] = b;
    // gate masks in local-bit coordinates, indexed by global gate index
    std::vector<uint64_t> lm(gates.size(), 0);
    for (int gi : ps.gates) {
        const PGate& g = gates[size_t(gi)];
        uint64_t m = uint64_t(1) << loc[g.p0];
        if (g.kind != QSV_G1Q) m |= uint64_t(1) << loc[g.p1];
        lm[size_t(gi)] = m;
    }
    const uint64_t canon = ((uint64_t(1) << K) - 1) & ~uint64_t(0xFF);   // local bits 8..K-1
    auto make_stage = [&](uint64_t S, std::vector<int>&& g) {
        Stage st;
        st.nr = RB;
        int j = 0;
        for (int b = 0; b < K && j < RB; ++b)
            if ((S >> b) & 1) st.rbits[j++] = b;
        // pad with the highest unused local bits
        for (int b = K - 1; b >= 0 && j < RB; --b)
            if (!((S >> b) & 1)) {
                S |= uint64_t(1) << b;
                st.rbits[j++] = b;
            }
        std::sort(st.rbits, st.rbits + RB);
        st.gates = std::move(g);
        return st;
    };

    std::vector<int> rem = ps.gates, take, defer;
    uint64_t S = canon;
    greedy(rem, lm, S, RB, true, take, defer);
    ps.stages.clear();
    ps.stages.push_back(make_stage(canon, std::move(take)));
    rem.swap(defer);
    std::vector<Stage> middle;
    while (!rem.empty()) {
        take.clear();
        defer.clear();
        S = 0;
        greedy(rem, lm, S, RB, false, take, defer);
        middle.push_back(make_stage(S, std::move(take)));
        rem.swap(defer);
    }
    if (middle.empty()) return;   // single stage: load, apply, store
    // the last middle stage becomes the canonical store stage if it fits
    Stage last;
    last.nr = RB;
    for (int j = 0; j < RB; ++j) last.rbits[j] = 8 + j;
    const Stage& lm_st = middle.back();
    uint64_t used = 0;
    for (int gi : lm_st.gates) used |= lm[size_t(gi)];
    if ((used & ~canon) == 0) {
        last.gates = lm_st.gates;
        middle.pop_back();
    }
    for (auto& m : middle) ps.stages.push_back(std::move(m));
    ps.stages.push_back(std::move(last));
}

std::vector<Pass> plan_passes(int n, const std::vector<PGate>& gates, const TileConfig& cfg) {
    std::vector<Pass> passes;
    std::vector<uint64_t> masks(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) masks[i] = gate_mask(gates[i]);
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
    const int K = std::min(cfg.tile_bits, n);
    const int L = std::min(cfg.low_bits, K);
    std::vector<int> rem(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) rem[i] = int(i);

    while (!rem.empty()) {
        uint64_t S = (uint64_t(1) << L) - 1;
        std::vector<int> take, defer;
        take.reserve(rem.size());
        greedy(rem, masks, S, K, false, take, defer);
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

}  // namespace qsv
