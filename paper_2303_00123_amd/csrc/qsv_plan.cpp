// Fusion planner: groups a gate list into passes.  Each pass covers a set S
// of index-bit positions (|S| = tile bits, always containing the lowest
// `low_bits` positions so every tile is made of contiguous runs); every gate
// of the pass acts only on positions in S, so one HBM read and one HBM write
// of the state apply the whole group.
//
// Ordering: gates are scanned in circuit order.  A gate joins the current
// pass if its positions fit in S (growing S while room is left) and none of
// its positions is "blocked"; a gate that cannot join is deferred and blocks
// its positions for the rest of the scan, so no later gate on those qubits
// can overtake it.  Gates that do join therefore only overtake deferred
// gates on disjoint qubits, with which they commute.
#include <algorithm>

#include "qsv_internal.h"

namespace qsv {

static inline uint64_t gate_mask(const PGate& g) {
    uint64_t m = uint64_t(1) << g.p0;
    if (g.kind != QSV_G1Q) m |= uint64_t(1) << g.p1;
    return m;
}

std::vector<Pass> plan_passes(int n, const std::vector<PGate>& gates, const TileConfig& cfg) {
    std::vector<Pass> passes;
    const int K = std::min(cfg.tile_bits, n);
    const int L = std::min(cfg.low_bits, K);
    std::vector<int> rem(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) rem[i] = int(i);

    while (!rem.empty()) {
        uint64_t S = (L >= 64) ? ~uint64_t(0) : ((uint64_t(1) << L) - 1);
        int cnt = L;
        uint64_t blocked = 0;
        std::vector<int> take, defer;
        take.reserve(rem.size());
        for (int gi : rem) {
            const uint64_t gm = gate_mask(gates[gi]);
            if (gm & blocked) {
                defer.push_back(gi);
                blocked |= gm;
                continue;
            }
            const uint64_t need = gm & ~S;
            const int add = __builtin_popcountll(need);
            if (cnt + add <= K) {
                S |= need;
                cnt += add;
                take.push_back(gi);
            } else {
                defer.push_back(gi);
                blocked |= gm;
            }
        }
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
        passes.push_back(std::move(ps));
        rem.swap(defer);
    }
    return passes;
}

}  // namespace qsv
