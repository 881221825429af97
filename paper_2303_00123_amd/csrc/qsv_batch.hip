// Batched persistent launch: many independent circuits (different qubit
// counts, gates and angles) in one kernel launch.
//
// Every circuit is planned like a single state (fused tile passes of 2^K
// amplitudes, register stages, gate fusion); a circuit narrower than K
// qubits is padded with idle qubits at the low index bits, so its whole
// state is one tile.  The launch processes a work list of items (circuit,
// pass, tile) that workgroups claim with an atomic counter:
//   * a circuit's first pass builds |0...0> in registers instead of loading;
//   * its last pass reduces sum_t w_t <Z^{m_t}> over the tile (FP64) instead
//     of storing the state; the workgroup finishing the circuit's last tile
//     adds the per-tile partials in tile order and writes out[b];
//   * a single-tile circuit (first == last pass) never touches HBM.
// Items are listed pass-level-major, so an item of pass p only ever waits
// for items of pass p-1 of its circuit, all of which were claimed earlier by
// running workgroups: the wait always ends, whatever the number of resident
// workgroups.  Waits are still bounded: past a spin limit the kernel raises
// an error flag and drains the queue without computing.
//
// HBM states of different circuits never alias; cross-workgroup visibility
// (the per-XCD L2s are not coherent with each other) uses agent-scope
// release/acquire on the per-circuit completion counters.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <map>
#include <string>
#include <thread>

#include "qsv_tile_core.h"

namespace qsv {
namespace {

using namespace tile;

enum { BP_FIRST = 1, BP_LAST = 2 };

struct BCirc {
    uint64_t state_off;   // amplitude offset of the circuit's state (multi-pass circuits)
    uint64_t part_off;    // offset of its per-tile partial sums
    int32_t tiles;        // tiles per pass
    int32_t npasses;
    int32_t term_beg, term_end;
};

struct BPass {
    int32_t circ;
    int32_t level;
    uint32_t rec_off;     // byte offset of the pass record in the plan
    int32_t flags;
};

struct BItem {
    int32_t pass;
    int32_t tile;
};

// counters layout (uint32): [0] next item, [1] error flag, [2 ..) done per circuit
constexpr int kCtrDone = 2;
// batches of at least this many circuits run as two parts (see qsv_batch_run)
constexpr int kSplitCircuits = 32;

__device__ __forceinline__ double zsign_sum(uint64_t x, const uint64_t* __restrict__ m,
                                            const double* __restrict__ w, int beg, int end) {
    double d = 0.0;
    for (int t = beg; t < end; ++t) d += (__popcll(x & m[t]) & 1) ? -w[t] : w[t];
    return d;
}

template <typename R, int K>
__global__ __launch_bounds__(kThreads) void k_batch(typename V2T<R>::type* __restrict__ states,
                                                    const char* __restrict__ plan,
                                                    const BCirc* __restrict__ circs,
                                                    const BPass* __restrict__ passes,
                                                    const BItem* __restrict__ items, int nitems,
                                                    const uint64_t* __restrict__ tmask,
                                                    const double* __restrict__ tw,
                                                    unsigned* __restrict__ ctr,
                                                    double* __restrict__ partials,
                                                    double* __restrict__ out, unsigned spin_limit) {
    using V = typename V2T<R>::type;
    constexpr bool SPLIT = K >= 13;   // as planned by build_batch
    constexpr int E = SPLIT ? 1 << (K - 1) : 1 << K;
    constexpr int RB = K - 8;
    constexpr int P = 1 << RB;
    __shared__ V tile[E];
    __shared__ double red[1][kThreads];
    __shared__ int s_item;
    __shared__ int s_flag;
    char* lds = reinterpret_cast<char*>(tile);
    const uint32_t tid = threadIdx.x;

    for (;;) {
        if (tid == 0) s_item = int(atomicAdd(&ctr[0], 1u));
        __syncthreads();
        // the same for every lane: scalar loads and registers for the item's tables
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= nitems) return;   // uniform: every wave of the workgroup leaves
        const BItem I = items[it];
        const BPass Pp = passes[I.pass];
        const BCirc C = circs[Pp.circ];
        const TPassHdr* hdr = reinterpret_cast<const TPassHdr*>(plan + Pp.rec_off);
        const int nst = hdr->nstages;
        const TStage* stg = reinterpret_cast<const TStage*>(plan + Pp.rec_off + sizeof(TPassHdr));
        const TGate<R>* gates = reinterpret_cast<const TGate<R>*>(
            plan + Pp.rec_off + sizeof(TPassHdr) + size_t(nst) * sizeof(TStage));

        uint64_t b = uint32_t(I.tile);
#pragma unroll
        for (int i = 0; i < K; ++i) b = insert0(b, hdr->pos[i]);
        const uint64_t xt = b | deposit(tid, hdr->tpos_ld, 8);   // register slot 0 (load mapping)
        V* const sp = states + C.state_off + xt;

        V v[P];
        bool ok = true;
        if (Pp.flags & BP_FIRST) {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                v[u].x = (xt | hdr->du[u]) == 0 ? R(1) : R(0);
                v[u].y = R(0);
            }
        } else {
            // wait until every tile of the circuit's previous pass is stored
            if (tid == 0) {
                const unsigned need = unsigned(Pp.level) * unsigned(C.tiles);
                unsigned spins = 0;
                int flag = 0;
                while (__hip_atomic_load(&ctr[kCtrDone + Pp.circ], __ATOMIC_ACQUIRE,
                                         __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (__hip_atomic_load(&ctr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                        ++spins > spin_limit) {
                        atomicOr(&ctr[1], 1u);
                        flag = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                s_flag = flag;
            }
            __syncthreads();
            ok = s_flag == 0;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (ok) {
#pragma unroll
                for (int u = 0; u < P; ++u) v[u] = ld_nt(sp + hdr->du[u]);
            }
        }
        if (ok) run_stages<R, K, K - 8, SPLIT>(v, lds, stg, nst, gates, tid);
        // store mapping, computed after the stages so it is not live across them
        const uint64_t xs = b | deposit(tid, hdr->tpos_st, 8);   // register slot 0
        V* const sq = states + C.state_off + xs;

        if (Pp.flags & BP_LAST) {
            double acc = 0.0;
            if (ok) {
#pragma unroll
                for (int u = 0; u < P; ++u) {
                    const double re = double(v[u].x), im = double(v[u].y);
                    acc += (re * re + im * im) *
                           zsign_sum(xs | hdr->du_st[u], tmask, tw, C.term_beg, C.term_end);
                }
            }
            red[0][tid] = acc;
            double tot[1];
            block_tree256<1>(red, tot);
            if (tid == 0) {
                if (C.tiles == 1 && C.npasses == 1) {
                    out[Pp.circ] = tot[0];
                } else {
                    partials[C.part_off + uint32_t(I.tile)] = tot[0];
                    const unsigned total = unsigned(C.npasses) * unsigned(C.tiles);
                    const unsigned prev = __hip_atomic_fetch_add(&ctr[kCtrDone + Pp.circ], 1u,
                                                                 __ATOMIC_ACQ_REL,
                                                                 __HIP_MEMORY_SCOPE_AGENT);
                    if (prev + 1 == total) {   // last tile of the circuit: fixed-order sum
                        double s = 0.0;
                        for (int t = 0; t < C.tiles; ++t) s += partials[C.part_off + t];
                        out[Pp.circ] = s;
                    }
                }
            }
        } else {
            if (ok) {
#pragma unroll
                for (int u = 0; u < P; ++u) st_nt(sq + hdr->du_st[u], v[u]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0)
                __hip_atomic_fetch_add(&ctr[kCtrDone + Pp.circ], 1u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();   // s_item / LDS reuse by the next item
    }
}

// zero n words (a kernel rather than a memset, so the sequence can be captured)
__global__ void k_zero(unsigned* __restrict__ p, size_t n) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

inline int pos_in(int n, int q) { return n - 1 - q; }

struct BatchBuild {
    // pass records are written later, straight into the upload buffer
    // (write_batch_records): per circuit its lowered gates and pass list
    // (an entry of the plan memo, or `own`), and per pass its record offset
    int dtype = 0;
    size_t plan_bytes = 0;
    std::vector<std::vector<PGate>> lowered;
    std::vector<std::vector<Pass>> own;
    std::vector<std::vector<Pass>*> plans;
    std::vector<size_t> rec_first;   // per circuit: index of its first pass in `passes`
    std::vector<BCirc> circs;
    std::vector<BPass> passes;
    std::vector<BItem> items;
    std::vector<uint64_t> tmask;
    std::vector<double> tw;
    uint64_t state_amps = 0;
    uint64_t partial_count = 0;
    uint64_t shape_key = 1469598103934665603ull;
};

void mix(uint64_t& h, uint64_t v) {
    for (int i = 0; i < 8; ++i) {
        h ^= (v >> (8 * i)) & 0xff;
        h *= 1099511628211ull;
    }
}

// f(0 .. n-1) on up to 16 host threads, the context's worker pool and the
// caller (work handed out one index at a time); serial for small n.  False if f threw (out of host memory): the
// exception stops at the worker instead of ending the process.
template <typename F>
bool parallel_for(qsv_ctx ctx, int n, F&& f) {
    std::atomic<bool> ok{true};
    auto guarded = [&](int i) {
        try {
            f(i);
        } catch (...) {
            ok = false;
        }
    };
    const unsigned hw = std::thread::hardware_concurrency();
    const int nt = std::min(int(hw ? hw : 1), 16);
    if (nt > 1 && n >= 8 && !ctx->pool) ctx->pool = pool_create(nt - 1);
    if (nt <= 1 || n < 8 || !ctx->pool) {
        for (int i = 0; i < n; ++i) guarded(i);
        return ok;
    }
    using G = decltype(guarded);
    const bool ran = pool_run(ctx->pool, n, [](void* a, int i) { (*static_cast<G*>(a))(i); }, &guarded);
    return ran && ok;
}

// A pass of one gate (or none) would run as an unfused kernel in the
// single-state path; here every pass is a tile pass, so it gets register
// stages like any other.
void make_single_stage(Pass& ps, const std::vector<PGate>& gates, int K, bool split) {
    ps.single = false;
    ps.rb = K - 8;
    ps.split = split;
    plan_pass_stages(ps.k, gates, ps);
}

// Plan every circuit and lay out the device tables.  Returns an error text
// on invalid input ("" on success).
std::string build_batch(qsv_ctx ctx, int nb, const int* nq, const int64_t* gate_off, const qsv_gate* g,
                        const double* params, int64_t nparams, const int64_t* term_off,
                        const uint64_t* qmasks, const double* w, int dtype, int K, int L,
                        BatchBuild& B, std::vector<PlanMemo>* memo) {
    const size_t amp = amp_bytes(dtype);
    B.dtype = dtype;
    // per-circuit pass lists: entries of the memo when there is one (reused
    // in place; the one-gate stage fix-up below is idempotent), else local
    std::vector<std::vector<Pass>>& own = B.own;
    std::vector<std::vector<Pass>*>& plans = B.plans;
    own.assign(static_cast<size_t>(memo ? 0 : nb), {});
    plans.assign(static_cast<size_t>(nb), nullptr);
    if (memo && memo->size() < size_t(nb)) memo->resize(size_t(nb));
    std::vector<std::vector<PGate>>& lowered = B.lowered;
    lowered.assign(static_cast<size_t>(nb), {});
    mix(B.shape_key, uint64_t(nb));
    mix(B.shape_key, uint64_t(dtype));
    // per circuit, in parallel: lower, fuse, plan (structure hash per circuit)
    std::vector<std::string> errs(static_cast<size_t>(nb));
    std::vector<uint64_t> chash(static_cast<size_t>(nb), 1469598103934665603ull);
    // 2^13-amplitude tiles (32 per thread) need the split exchange to fit
    // two workgroups per compute unit
    const TileConfig bcfg{K, L, K - 8, coal_bits_for(dtype), K >= 13 ? 1 : 0};
    const bool built = parallel_for(ctx, nb, [&](int c) {
        const int n = nq[c];
        const int ne = n < K ? K : n;
        const int64_t g0 = gate_off[c], g1 = gate_off[c + 1];
        // built in locals: the per-circuit slots of `lowered` and `chash` sit
        // side by side, and writing them per gate from several threads
        // bounced their cache lines between cores
        std::vector<PGate> low;
        low.reserve(size_t(g1 - g0));
        uint64_t h = chash[size_t(c)];
        for (int64_t i = g0; i < g1; ++i) {
            const qsv_gate& G = g[i];
            PGate p{};
            auto err = [&](const char* what) {
                errs[size_t(c)] = "circuit " + std::to_string(c) + " gate " + std::to_string(i - g0) + ": " + what;
            };
            const bool two = G.kind == QSV_GC1Q || G.kind == QSV_G2Q;
            if (G.kind < QSV_G1Q || G.kind > QSV_GROT) return err("unknown kind");
            if (G.cmask || G.cvals) return err("extra controls are not supported in a batch");
            if (G.q0 < 0 || G.q0 >= n || (two && (G.q1 < 0 || G.q1 >= n || G.q1 == G.q0)))
                return err("bad qubit");
            mix(h, uint64_t(G.kind) | (uint64_t(G.q0) << 8) | (uint64_t(two ? G.q1 : 0) << 16) |
                       (uint64_t(G.ctrl_state & 1) << 24) | (uint64_t(G.axis & 3) << 26));
            p.kind = G.kind == QSV_GROT ? QSV_G1Q : G.kind;
            p.p0 = pos_in(ne, G.q0);
            p.p1 = two ? pos_in(ne, G.q1) : 0;
            p.cs = G.ctrl_state;
            if (G.kind == QSV_GC1Q && G.ctrl_state != 0 && G.ctrl_state != 1) return err("bad control state");
            if (G.kind == QSV_GROT) {
                if (G.axis < 0 || G.axis > 2) return err("bad axis");
                if (G.param < 0 || G.param >= nparams) return err("parameter index out of range");
                rotation_matrix(G.axis, params[G.param], p.m);
            } else {
                std::memcpy(p.m, G.m, sizeof(double) * (G.kind == QSV_G2Q ? 32 : 8));
            }
            low.push_back(p);
        }
        chash[size_t(c)] = h;
        std::vector<PGate>& pg = lowered[size_t(c)];
        pg = prefuse(low);
        if (memo) {
            PlanMemo& m = (*memo)[size_t(c)];
            plan_memo(m, ne, pg, bcfg);   // same structure: same plan
            plans[size_t(c)] = &m.passes;
        } else {
            own[size_t(c)] = plan_passes(ne, pg, bcfg);
            plans[size_t(c)] = &own[size_t(c)];
        }
        std::vector<Pass>& pl = *plans[size_t(c)];
        if (pl.empty()) {
            // no gates: still one (empty) pass to produce the observable
            Pass ps;
            ps.k = K;
            ps.rb = K - 8;
            ps.coal = bcfg.coal_bits;
            for (int b = 0; b < K; ++b) ps.pos[b] = b;
            pl.push_back(ps);
        }
        // a pass of one gate would run as an unfused kernel in the
        // single-state path; here every pass is a tile pass
        for (Pass& ps : pl)
            if (ps.single || ps.stages.empty()) make_single_stage(ps, pg, K, bcfg.split != 0);
    });
    if (!built) return "out of host memory while planning";
    for (int c = 0; c < nb; ++c)
        if (!errs[size_t(c)].empty()) return errs[size_t(c)];
    for (int c = 0; c < nb; ++c) mix(B.shape_key, chash[size_t(c)]);
    int maxp = 0;
    for (int c = 0; c < nb; ++c) {
        const int n = nq[c];
        const int ne = n < K ? K : n;
        BCirc bc{};
        bc.tiles = int32_t(uint64_t(1) << (ne - K));
        bc.npasses = int32_t(plans[size_t(c)]->size());
        bc.term_beg = int32_t(B.tmask.size());
        for (int64_t t = term_off[c]; t < term_off[c + 1]; ++t) {
            if (n < 64 && (qmasks[t] >> n)) return "circuit " + std::to_string(c) + ": term names a qubit >= n";
            uint64_t pm = 0;
            for (int q = 0; q < n; ++q)
                if ((qmasks[t] >> q) & 1) pm |= uint64_t(1) << pos_in(ne, q);
            B.tmask.push_back(pm);
            B.tw.push_back(w ? w[t] : 1.0);
            mix(B.shape_key, qmasks[t]);
        }
        bc.term_end = int32_t(B.tmask.size());
        if (bc.npasses > 1 || bc.tiles > 1) {
            bc.state_off = B.state_amps;
            B.state_amps += uint64_t(1) << ne;
        }
        bc.part_off = B.partial_count;
        B.partial_count += uint64_t(bc.tiles);
        B.circs.push_back(bc);
        if (bc.npasses > maxp) maxp = bc.npasses;
    }
    // pass records: offsets in order (written later by write_batch_records)
    std::vector<size_t>& rec_first = B.rec_first;
    rec_first.assign(static_cast<size_t>(nb) + 1, 0);
    {
        size_t total = 0;
        for (int c = 0; c < nb; ++c) {
            const std::vector<Pass>& pl = *plans[size_t(c)];
            rec_first[size_t(c)] = B.passes.size();
            for (size_t p = 0; p < pl.size(); ++p) {
                BPass bp{};
                bp.circ = c;
                bp.level = int32_t(p);
                bp.rec_off = uint32_t(total);
                bp.flags = (p == 0 ? BP_FIRST : 0) | (p + 1 == pl.size() ? BP_LAST : 0);
                B.passes.push_back(bp);
                total += pass_record_bytes(dtype, pl[p]);
            }
        }
        rec_first[size_t(nb)] = B.passes.size();
        if (total >= (size_t(1) << 32)) return "batch plan too large";
        B.plan_bytes = total;
    }
    // items, pass-level-major; within a level, larger circuits first
    std::vector<int> pass_first(static_cast<size_t>(nb), 0);
    {
        int k = 0;
        for (int c = 0; c < nb; ++c) {
            pass_first[size_t(c)] = k;
            k += B.circs[size_t(c)].npasses;
        }
    }
    std::vector<int> order(static_cast<size_t>(nb));
    for (int c = 0; c < nb; ++c) order[size_t(c)] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b2) {
        return B.circs[size_t(a)].tiles > B.circs[size_t(b2)].tiles;
    });
    {
        size_t nitems = 0;
        for (const BCirc& bc : B.circs) nitems += size_t(bc.npasses) * size_t(bc.tiles);
        B.items.reserve(nitems);
    }
    for (int lv = 0; lv < maxp; ++lv)
        for (int c : order) {
            const BCirc& bc = B.circs[size_t(c)];
            if (lv >= bc.npasses) continue;
            for (int t = 0; t < bc.tiles; ++t) B.items.push_back(BItem{pass_first[size_t(c)] + lv, t});
        }
    (void)amp;
    return "";
}

// The pass records of a built batch, written in parallel at dst (plan_bytes
// bytes; each record is cleared first, so padding is deterministic).
// QSV_ERR_NOMEM if a worker ran out of host memory, QSV_ERR_INTERNAL on a
// planner inconsistency.
qsv_status write_batch_records(qsv_ctx ctx, const BatchBuild& B, char* dst) {
    const int nb = int(B.plans.size());
    std::atomic<bool> bad{false};
    const bool written = parallel_for(ctx, nb, [&](int c) {
        const std::vector<Pass>& pl = *B.plans[size_t(c)];
        for (size_t p = 0; p < pl.size(); ++p) {
            const size_t i = B.rec_first[size_t(c)] + p;
            const size_t off = B.passes[i].rec_off;
            const size_t end = i + 1 < B.passes.size() ? B.passes[i + 1].rec_off : B.plan_bytes;
            std::memset(dst + off, 0, end - off);
            if (!write_pass_record(B.dtype, dst + off, B.lowered[size_t(c)], pl[p])) bad = true;
        }
    });
    if (!written) return QSV_ERR_NOMEM;
    return bad ? QSV_ERR_INTERNAL : QSV_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t plan, circs, passes, items, tmask, tw, total;
};

Layout upload_layout(const BatchBuild& B) {
    Layout L{};
    size_t o = 0;
    L.plan = o; o = align256(o + B.plan_bytes);
    L.circs = o; o = align256(o + B.circs.size() * sizeof(BCirc));
    L.passes = o; o = align256(o + B.passes.size() * sizeof(BPass));
    L.items = o; o = align256(o + B.items.size() * sizeof(BItem));
    L.tmask = o; o = align256(o + (B.tmask.size() + 1) * sizeof(uint64_t));
    L.tw = o; o = align256(o + (B.tw.size() + 1) * sizeof(double));
    L.total = o;
    return L;
}

template <typename R, int K>
hipError_t launch_batch(qsv_ctx ctx, hipStream_t stream, const char* dev, const Layout& L,
                        int nb, int nitems, void* states, unsigned* ctr, double* partials,
                        double* out) {
    using V = typename V2T<R>::type;
    static int per_cu = 0;
    if (per_cu == 0) {
        int nbk = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nbk, k_batch<R, K>, kThreads, 0) !=
                hipSuccess || nbk < 1)
            nbk = 1;
        per_cu = nbk;
    }
    unsigned grid = unsigned(per_cu) * unsigned(ctx->num_cus);
    if (grid > unsigned(nitems)) grid = unsigned(nitems);
    if (grid == 0) grid = 1;
    // x s_sleep(8): about 2 s before giving up; QSV_BATCH_SPIN_LIMIT overrides
    // it (0 makes every wait that has to wait fail at once, so tests can drive
    // the error path with every workgroup still exiting normally)
    unsigned spin_limit = 1u << 22;
    if (const char* sl = std::getenv("QSV_BATCH_SPIN_LIMIT"))
        spin_limit = unsigned(std::strtoul(sl, nullptr, 10));
    hipLaunchKernelGGL((k_batch<R, K>), dim3(grid), dim3(kThreads), 0, stream,
                       static_cast<V*>(states), dev + L.plan,
                       reinterpret_cast<const BCirc*>(dev + L.circs),
                       reinterpret_cast<const BPass*>(dev + L.passes),
                       reinterpret_cast<const BItem*>(dev + L.items), nitems,
                       reinterpret_cast<const uint64_t*>(dev + L.tmask),
                       reinterpret_cast<const double*>(dev + L.tw), ctr, partials, out, spin_limit);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_k(qsv_ctx ctx, hipStream_t stream, int K, const char* dev, const Layout& L,
                          int nb, int nitems, void* states, unsigned* ctr, double* partials,
                          double* out) {
    switch (K) {
    case 10: return launch_batch<R, 10>(ctx, stream, dev, L, nb, nitems, states, ctr, partials, out);
    case 11: return launch_batch<R, 11>(ctx, stream, dev, L, nb, nitems, states, ctr, partials, out);
    case 12: return launch_batch<R, 12>(ctx, stream, dev, L, nb, nitems, states, ctr, partials, out);
    case 13:
        // complex128 at 2^13: two 32-amplitude register sets leave no room
        // for the batch bookkeeping within 256 registers
        if constexpr (sizeof(R) == 4)
            return launch_batch<R, 13>(ctx, stream, dev, L, nb, nitems, states, ctr, partials, out);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// ---------------------------------------------------------------- driver
struct BatchRun {
    Layout L;
    size_t ctr_words = 0, partial_count = 0, state_bytes = 0;
    int nitems = 0;
};

// Enqueue one part of a batch (upload, counter reset, kernel, result
// download) on `stream`, with slot b's buffers (grown on demand beforehand).
static hipError_t enqueue_batch(qsv_ctx ctx, BatchSlot& b, hipStream_t stream, int dtype, int K, int nb,
                                const BatchRun& R) {
    char* dev = static_cast<char*>(b.d);
    hipError_t e = hipMemcpyAsync(dev, b.h, R.L.total, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    unsigned* ctr = reinterpret_cast<unsigned*>(dev + b.ctr_off);
    double* out = reinterpret_cast<double*>(dev + b.out_off);
    double* partials = reinterpret_cast<double*>(dev + b.part_off);
    void* states = dev + b.state_off;
    const size_t zw = R.ctr_words;   // item counter, error flag, per-circuit completion counts
    hipLaunchKernelGGL(k_zero, dim3(unsigned((zw + 255) / 256)), dim3(256), 0, stream, ctr, zw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_before_on(ctx, stream, dtype == QSV_C128 ? "batch_c128" : "batch_c64", 0.0);
    e = dtype == QSV_C128
            ? launch_batch_k<double>(ctx, stream, K, dev, R.L, nb, R.nitems, states, ctr, partials, out)
            : launch_batch_k<float>(ctx, stream, K, dev, R.L, nb, R.nitems, states, ctr, partials, out);
    prof_after_on(ctx, stream);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(b.h_out, out, sizeof(double) * (size_t(nb) + 1), hipMemcpyDeviceToHost, stream);
}

// Plan and stage nb circuits into slot b for tile shape (K, L); sizes the
// slot's buffers.
static qsv_status stage_batch(qsv_ctx ctx, BatchSlot& b, int nb, const int* nq, const int64_t* gate_off,
                              const qsv_gate* g, const double* params, int64_t nparams,
                              const int64_t* term_off, const uint64_t* qmasks, const double* w,
                              int dtype, int K, int L, BatchRun& R, uint64_t& key) {
    BatchBuild B;
    const auto t0 = std::chrono::steady_clock::now();
    std::string err = build_batch(ctx, nb, nq, gate_off, g, params, nparams, term_off, qmasks, w, dtype,
                                  K, L, B, &b.memo);
    const auto t1 = std::chrono::steady_clock::now();
    if (!err.empty()) {
        ctx->last_error = "qsv_batch_run: " + err;
        return QSV_ERR_ARG;
    }
    key = B.shape_key;
    R.L = upload_layout(B);
    R.nitems = int(B.items.size());
    R.ctr_words = size_t(kCtrDone) + size_t(nb);
    R.partial_count = B.partial_count;
    R.state_bytes = B.state_amps * amp_bytes(dtype);
    // device buffer: [upload | counters | out | partials | states]
    const size_t ctr_off = R.L.total;
    const size_t out_off = align256(ctr_off + R.ctr_words * sizeof(unsigned));
    const size_t part_off = align256(out_off + (size_t(nb) + 1) * sizeof(double));
    const size_t state_off = align256(part_off + (R.partial_count + 1) * sizeof(double));
    const size_t need = state_off + R.state_bytes + 256;
    if (need > b.d_bytes || R.L.total > b.h_bytes || size_t(nb) + 1 > b.h_out_n) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess && ctx->batch_stream) e = hipStreamSynchronize(ctx->batch_stream);
        if (e != hipSuccess) {
            ctx->last_error = std::string("qsv_batch_run: ") + hipGetErrorString(e);
            return QSV_ERR_HIP;
        }
        if (b.graph_exec) {
            hipGraphExecDestroy(static_cast<hipGraphExec_t>(b.graph_exec));
            b.graph_exec = nullptr;
            b.graph_key = 0;
        }
        if (need > b.d_bytes) {
            if (b.d) hipFree(b.d);
            b.d = nullptr;
            b.d_bytes = 0;
            if (hipMalloc(&b.d, need) != hipSuccess) {
                (void)hipGetLastError();
                ctx->last_error = "qsv_batch_run: device allocation of " + std::to_string(need) + " bytes failed";
                return QSV_ERR_NOMEM;
            }
            b.d_bytes = need;
        }
        if (R.L.total > b.h_bytes) {
            if (b.h) hipHostFree(b.h);
            b.h = nullptr;
            b.h_bytes = 0;
            if (hipHostMalloc(&b.h, R.L.total, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                ctx->last_error = "qsv_batch_run: pinned allocation failed";
                return QSV_ERR_NOMEM;
            }
            b.h_bytes = R.L.total;
        }
        if (size_t(nb) + 1 > b.h_out_n) {
            if (b.h_out) hipHostFree(b.h_out);
            b.h_out = nullptr;
            b.h_out_n = 0;
            if (hipHostMalloc(reinterpret_cast<void**>(&b.h_out), sizeof(double) * (size_t(nb) + 1),
                              hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                ctx->last_error = "qsv_batch_run: pinned allocation failed";
                return QSV_ERR_NOMEM;
            }
            b.h_out_n = size_t(nb) + 1;
        }
    }
    b.ctr_off = ctr_off;
    b.out_off = out_off;
    b.part_off = part_off;
    b.state_off = state_off;
    char* h = static_cast<char*>(b.h);
    if (qsv_status ws = write_batch_records(ctx, B, h + R.L.plan)) {
        ctx->last_error = ws == QSV_ERR_NOMEM ? "qsv_batch_run: out of host memory while writing records"
                                              : "qsv_batch_run: internal planner error";
        return ws;
    }
    std::memcpy(h + R.L.circs, B.circs.data(), B.circs.size() * sizeof(BCirc));
    std::memcpy(h + R.L.passes, B.passes.data(), B.passes.size() * sizeof(BPass));
    std::memcpy(h + R.L.items, B.items.data(), B.items.size() * sizeof(BItem));
    if (!B.tmask.empty()) std::memcpy(h + R.L.tmask, B.tmask.data(), B.tmask.size() * sizeof(uint64_t));
    if (!B.tw.empty()) std::memcpy(h + R.L.tw, B.tw.data(), B.tw.size() * sizeof(double));
    if (log_enabled()) {
        const auto t2 = std::chrono::steady_clock::now();
        logf("batch staging: %d circuits, %d items, tile 2^%d low %d, build %.2f ms, records and copies %.2f ms",
             nb, R.nitems, K, L, std::chrono::duration<double, std::milli>(t1 - t0).count(),
             std::chrono::duration<double, std::milli>(t2 - t1).count());
    }
    return QSV_OK;
}

// Wait for `stream`; check a part's error flag.
static qsv_status wait_batch(qsv_ctx ctx, hipStream_t stream) {
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        ctx->last_error = std::string("qsv_batch_run: ") + hipGetErrorName(e) + " " + hipGetErrorString(e);
        return QSV_ERR_HIP;
    }
    return QSV_OK;
}
static qsv_status check_batch(qsv_ctx ctx, const BatchSlot& b) {
    unsigned flag = 0;
    const hipError_t e = hipMemcpy(&flag, static_cast<const char*>(b.d) + b.ctr_off + sizeof(unsigned),
                                   sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e != hipSuccess || flag) {
        ctx->last_error = "qsv_batch_run: a dependency wait exceeded its spin limit";
        return QSV_ERR_HIP;
    }
    return QSV_OK;
}

// Launch a staged part on `stream`: its captured graph (captured anew when
// anything it bakes in changed) or the eager sequence.
static hipError_t launch_part(qsv_ctx ctx, BatchSlot& b, hipStream_t stream, bool graph, int dtype, int K,
                              int L, int nb, const BatchRun& R, uint64_t key) {
    if (!graph) return enqueue_batch(ctx, b, stream, dtype, K, nb, R);
    // everything the captured graph bakes in: tile shape, upload layout,
    // item count (grid), counter words, buffer offsets and sizes -- new
    // angles can change fused gates and pass counts, so the shape key
    // alone does not fix them
    uint64_t gkey = key;
    for (uint64_t v : {uint64_t(K), uint64_t(L), uint64_t(R.L.plan), uint64_t(R.L.circs),
                       uint64_t(R.L.passes), uint64_t(R.L.items), uint64_t(R.L.tmask),
                       uint64_t(R.L.tw), uint64_t(R.L.total), uint64_t(R.nitems),
                       uint64_t(R.ctr_words), uint64_t(R.partial_count), uint64_t(R.state_bytes),
                       uint64_t(b.ctr_off), uint64_t(b.out_off), uint64_t(b.part_off), uint64_t(b.state_off),
                       reinterpret_cast<uint64_t>(b.d), reinterpret_cast<uint64_t>(b.h),
                       reinterpret_cast<uint64_t>(b.h_out)})
        mix(gkey, v);
    hipError_t e = hipSuccess;
    if (!b.graph_exec || b.graph_key != gkey) {
        // capture from an idle stream (an earlier part may still run on it)
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        if (b.graph_exec) {
            hipGraphExecDestroy(static_cast<hipGraphExec_t>(b.graph_exec));
            b.graph_exec = nullptr;
        }
        hipGraph_t gr = nullptr;
        e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const bool prof = ctx->profiling;
            ctx->profiling = false;   // no event records inside the graph
            const hipError_t e2 = enqueue_batch(ctx, b, stream, dtype, K, nb, R);
            ctx->profiling = prof;
            e = hipStreamEndCapture(stream, &gr);
            if (e2 != hipSuccess) e = e2;
        }
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
        if (gr) hipGraphDestroy(gr);
        if (e != hipSuccess) return e;
        b.graph_exec = exec;
        b.graph_key = gkey;
    }
    prof_before_on(ctx, stream, dtype == QSV_C128 ? "batch_graph_c128" : "batch_graph_c64", 0.0);
    e = hipGraphLaunch(static_cast<hipGraphExec_t>(b.graph_exec), stream);
    prof_after_on(ctx, stream);
    return e;
}

// Key of a batch's shape: qubit counts, gate kinds / qubits / control states /
// axes and observable masks -- everything but angles, matrices and weights.
// Words are mixed whole (one multiply each, not one per byte): the key is
// computed on every call, over every gate of the batch.
static uint64_t shape_key(int nb, const int* nq, const int64_t* gate_off, const qsv_gate* g,
                          const int64_t* term_off, const uint64_t* qmasks, int dtype) {
    uint64_t h = 1469598103934665603ull;
    auto wmix = [&h](uint64_t v) {
        h = (h ^ v) * 0x9e3779b97f4a7c15ull;
        h ^= h >> 29;
    };
    wmix(uint64_t(nb));
    wmix(uint64_t(dtype));
    for (int c = 0; c < nb; ++c) {
        wmix(uint64_t(nq[c]));
        for (int64_t i = gate_off[c]; i < gate_off[c + 1]; ++i) {
            const qsv_gate& G = g[i];
            wmix(uint64_t(uint32_t(G.kind)) | (uint64_t(uint32_t(G.q0)) << 8) |
                 (uint64_t(uint32_t(G.q1)) << 20) | (uint64_t(G.ctrl_state & 1) << 32) |
                 (uint64_t(G.axis & 3) << 33));
        }
        for (int64_t t = term_off[c]; t < term_off[c + 1]; ++t) wmix(qmasks[t]);
        wmix(0x5eedull);
    }
    return h;
}

// Tile shapes the autotuner tries for a batch, best first by default.
static const int kTuneShapes[][2] = {{13, 3}, {12, 3}, {11, 3}, {10, 2}, {13, 4}, {12, 4}, {11, 2}, {10, 3}};

}  // namespace qsv

using namespace qsv;

extern "C" qsv_status qsv_batch_run(qsv_ctx ctx, int nb, const int* nq, const int64_t* gate_off,
                                    const qsv_gate* g, const double* params, int64_t nparams,
                                    const int64_t* term_off, const uint64_t* qmasks,
                                    const double* w, int dtype, double* out, int flags) {
    try {
        if (!ctx) return QSV_ERR_ARG;
        const auto t_entry = std::chrono::steady_clock::now();
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
            ctx->last_error = "the context's device is not the current HIP device";
            return QSV_ERR_ARG;
        }
        if (dtype != QSV_C64 && dtype != QSV_C128) {
            ctx->last_error = "qsv_batch_run: dtype must be QSV_C64 or QSV_C128";
            return QSV_ERR_DTYPE;
        }
        if (nb < 1 || !nq || !gate_off || !term_off || !out || (nparams > 0 && !params) || nparams < 0) {
            ctx->last_error = "qsv_batch_run: bad arguments";
            return QSV_ERR_ARG;
        }
        if (flags & ~(QSV_FLAG_CAPTURE_GRAPH | QSV_FLAG_TUNE)) {
            ctx->last_error = "qsv_batch_run: unknown flag";
            return QSV_ERR_ARG;
        }
        for (int c = 0; c < nb; ++c) {
            if (nq[c] < 1 || nq[c] > kMaxBatchQubits) {
                ctx->last_error = "qsv_batch_run: circuit " + std::to_string(c) + " has " +
                                  std::to_string(nq[c]) + " qubits (allowed 1.." +
                                  std::to_string(kMaxBatchQubits) + ")";
                return QSV_ERR_SIZE;
            }
            if (gate_off[c + 1] < gate_off[c] || term_off[c + 1] < term_off[c]) {
                ctx->last_error = "qsv_batch_run: offsets must be non-decreasing";
                return QSV_ERR_ARG;
            }
        }
        if (gate_off[0] != 0 || term_off[0] != 0 || (gate_off[nb] > 0 && !g) || (term_off[nb] > 0 && !qmasks)) {
            ctx->last_error = "qsv_batch_run: bad offsets or arrays";
            return QSV_ERR_ARG;
        }
        // tile shape: the tuned choice for this batch shape, if any
        uint64_t key = 0;
        int K = dtype == QSV_C128 ? 12 : 13, L = dtype == QSV_C128 ? 3 : 4;
        {
            key = shape_key(nb, nq, gate_off, g, term_off, qmasks, dtype);
            qsv_status s = QSV_OK;
            int tk = 0, tl = 0;
            if (tune_lookup(ctx, key, dtype, &tk, &tl)) {
                K = tk;
                L = tl;
            } else if (flags & QSV_FLAG_TUNE) {
                // time each candidate twice and keep its faster run (every run
                // computes the full, correct batch)
                double best = 1e30;
                for (const auto& sh : kTuneShapes) {
                    if (sh[0] >= 13 && dtype == QSV_C128) continue;   // not compiled (see launch_batch_k)
                    uint64_t k2 = 0;
                    BatchRun Rc;
                    s = stage_batch(ctx, ctx->batch[0], nb, nq, gate_off, g, params, nparams, term_off, qmasks,
                                    w, dtype, sh[0], sh[1], Rc, k2);
                    if (s != QSV_OK) return s;
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
                        if (e0) hipEventDestroy(e0);
                        (void)hipGetLastError();
                        ctx->last_error = "qsv_batch_run: could not create the tuner's timing events";
                        return QSV_ERR_HIP;
                    }
                    float ms = 1e30f;
                    hipError_t e = hipSuccess;
                    for (int rep = 0; rep < 2 && e == hipSuccess && s == QSV_OK; ++rep) {
                        hipEventRecord(e0, ctx->stream);
                        e = enqueue_batch(ctx, ctx->batch[0], ctx->stream, dtype, sh[0], nb, Rc);
                        hipEventRecord(e1, ctx->stream);
                        if (e == hipSuccess) s = wait_batch(ctx, ctx->stream);
                        if (e == hipSuccess && s == QSV_OK) s = check_batch(ctx, ctx->batch[0]);
                        if (e == hipSuccess && s == QSV_OK)
                            std::memcpy(out, ctx->batch[0].h_out, sizeof(double) * size_t(nb));
                        float t = 0.f;
                        if (e == hipSuccess && s == QSV_OK && hipEventElapsedTime(&t, e0, e1) == hipSuccess &&
                            t < ms)
                            ms = t;
                    }
                    hipEventDestroy(e0);
                    hipEventDestroy(e1);
                    if (e != hipSuccess) {
                        ctx->last_error = std::string("qsv_batch_run: ") + hipGetErrorString(e);
                        return QSV_ERR_HIP;
                    }
                    if (s != QSV_OK) return s;
                    if (ms < best) {
                        best = ms;
                        K = sh[0];
                        L = sh[1];
                    }
                }
                tune_store(ctx, key, dtype, K, L, best);
            }
        }
        // Two parts when the batch is large enough: the second part is staged
        // on the host while the first one runs on the GPU.  Each part has its
        // own buffers, plan memo and captured graph; both run on one stream.
        const bool graph = (flags & QSV_FLAG_CAPTURE_GRAPH) != 0;
        hipStream_t stream = ctx->stream;
        if (graph) {
            if (!ctx->batch_stream) {
                if (hipStreamCreateWithFlags(&ctx->batch_stream, hipStreamNonBlocking) != hipSuccess) {
                    ctx->last_error = "qsv_batch_run: stream creation failed";
                    return QSV_ERR_HIP;
                }
            }
            stream = ctx->batch_stream;
            // order the batch after the context stream's earlier work
            const hipError_t e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) {
                ctx->last_error = std::string("qsv_batch_run: ") + hipGetErrorString(e);
                return QSV_ERR_HIP;
            }
        }
        // (three or four parts measured no faster: each launch adds a drain tail)
        const int parts = nb >= kSplitCircuits ? 2 : 1;
        const int first[3] = {0, parts == 2 ? nb / 2 : nb, nb};
        for (int p = 0; p < parts; ++p) {
            const int c0 = first[p], np = first[p + 1] - first[p];
            BatchRun R;
            uint64_t pkey = 0;
            qsv_status s = stage_batch(ctx, ctx->batch[p], np, nq + c0, gate_off + c0, g, params, nparams,
                                       term_off + c0, qmasks, w, dtype, K, L, R, pkey);
            if (s != QSV_OK) return s;
            const hipError_t e = launch_part(ctx, ctx->batch[p], stream, graph, dtype, K, L, np, R, pkey);
            if (e != hipSuccess) {
                ctx->last_error = std::string(graph ? "qsv_batch_run (graph): " : "qsv_batch_run: ") +
                                  hipGetErrorString(e);
                return QSV_ERR_HIP;
            }
        }
        const auto t_launched = std::chrono::steady_clock::now();
        if (qsv_status s = wait_batch(ctx, stream)) return s;
        for (int p = 0; p < parts; ++p)   // every part checked before out is written
            if (qsv_status s = check_batch(ctx, ctx->batch[p])) return s;
        for (int p = 0; p < parts; ++p)
            std::memcpy(out + first[p], ctx->batch[p].h_out, sizeof(double) * size_t(first[p + 1] - first[p]));
        if (log_enabled()) {
            const auto t_done = std::chrono::steady_clock::now();
            logf("batch call: %d part(s), %.2f ms to launch, %.2f ms waiting and reading results", parts,
                 std::chrono::duration<double, std::milli>(t_launched - t_entry).count(),
                 std::chrono::duration<double, std::milli>(t_done - t_launched).count());
        }
        return QSV_OK;
    } catch (const std::bad_alloc&) {
        return QSV_ERR_NOMEM;
    } catch (...) {
        return QSV_ERR_INTERNAL;
    }
}
