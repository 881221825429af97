// Fused tile pass: one workgroup loads a tile of 2^k amplitudes spanning the
// pass's k index-bit positions into LDS, applies every gate of the pass to
// it, and writes it back -- one HBM read and one HBM write for the whole
// gate group.  Tile t of the pass covers the indices whose non-tile bits
// spell t (zero-bit insertion at each tile position, ascending, generalising
// the masks of Sec. 2.1-2.2 from one or two positions to k).  Because the
// tile positions always include the lowest bits, each tile is a set of
// contiguous runs of at least 2^low_bits amplitudes.
//
// Inside the tile the gates use the same pair/quad index maps as the
// unfused kernels (Algs. 1-3), on local bit positions.
#include "qsv_common.h"
#include "qsv_internal.h"

namespace qsv {
namespace {

constexpr int kThreads = 256;

template <typename R>
struct TileK;
template <>
struct TileK<double> { static constexpr int value = 12; };   // 4096 x 16 B = 64 KiB
template <>
struct TileK<float> { static constexpr int value = 13; };    // 8192 x 8 B = 64 KiB

// Global offset of local element index e: deposit e's bits at pos[].
__device__ __forceinline__ uint64_t deposit(uint32_t e, const int32_t* pos, int k) {
    uint64_t off = 0;
    for (int i = 0; i < k; ++i)
        if ((e >> i) & 1u) off |= uint64_t(1) << pos[i];
    return off;
}

template <typename R, int KMAX>
__global__ __launch_bounds__(kThreads) void k_tile(typename V2T<R>::type* __restrict__ s,
                                                   const TPassHdr* __restrict__ hdr,
                                                   const TGate<R>* __restrict__ gates) {
    using V = typename V2T<R>::type;
    constexpr int EMAX = 1 << KMAX;
    constexpr int PER = EMAX / kThreads;   // elements per thread at k = KMAX
    __shared__ V tile[EMAX];

    const int k = hdr->k;
    const int ng = hdr->ngates;
    const uint32_t E = 1u << k;
    const uint32_t tid = threadIdx.x;

    // base index of this tile: insert a zero at every tile position
    uint64_t base = blockIdx.x;
    for (int i = 0; i < k; ++i) base = insert0(base, hdr->pos[i]);
    const int klo = k < 8 ? k : 8;
    const uint64_t dt = base | deposit(tid, hdr->pos, klo);

    // ---- load: element e = u*256 + tid
    {
        V buf[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t e = uint32_t(u) * kThreads + tid;
            if (e < E) {
                const uint64_t dm = deposit(uint32_t(u), hdr->pos + 8, k - 8 > 0 ? k - 8 : 0);
                buf[u] = s[dt | dm];
            }
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t e = uint32_t(u) * kThreads + tid;
            if (e < E) tile[e] = buf[u];
        }
    }
    __syncthreads();

    // ---- gates
    for (int g = 0; g < ng; ++g) {
        const TGate<R>& G = gates[g];
        const int kind = G.kind;
        if (kind == QSV_G1Q) {
            const int l = G.l0;
            const uint32_t w = 1u << l;
            constexpr int NP = EMAX / 2 / kThreads;
            V a[NP], b[NP];
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                const uint32_t j = uint32_t(u) * kThreads + tid;
                if (j < E / 2) {
                    const uint32_t ia = insert0_32(j, l);
                    a[u] = tile[ia];
                    b[u] = tile[ia + w];
                }
            }
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                const uint32_t j = uint32_t(u) * kThreads + tid;
                if (j < E / 2) {
                    const uint32_t ia = insert0_32(j, l);
                    V oa, ob;
                    mv2(G.m, a[u], b[u], oa, ob);
                    tile[ia] = oa;
                    tile[ia + w] = ob;
                }
            }
        } else if (kind == QSV_GC1Q) {
            const int lc = G.l0, lt = G.l1;
            const int llo = lc < lt ? lc : lt, lhi = lc < lt ? lt : lc;
            const uint32_t wt = 1u << lt;
            const uint32_t wc = G.cs ? (1u << lc) : 0u;
            constexpr int NP = EMAX / 4 / kThreads > 0 ? EMAX / 4 / kThreads : 1;
            V a[NP], b[NP];
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                const uint32_t j = uint32_t(u) * kThreads + tid;
                if (j < E / 4) {
                    const uint32_t ia = insert0_32(insert0_32(j, llo), lhi) | wc;
                    a[u] = tile[ia];
                    b[u] = tile[ia + wt];
                }
            }
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                const uint32_t j = uint32_t(u) * kThreads + tid;
                if (j < E / 4) {
                    const uint32_t ia = insert0_32(insert0_32(j, llo), lhi) | wc;
                    V oa, ob;
                    mv2(G.m, a[u], b[u], oa, ob);
                    tile[ia] = oa;
                    tile[ia + wt] = ob;
                }
            }
        } else {
            const int la = G.l0, lb = G.l1;
            const int llo = la < lb ? la : lb, lhi = la < lb ? lb : la;
            const uint32_t wa = 1u << la, wb = 1u << lb;
            constexpr int NQ = EMAX / 4 / kThreads > 0 ? EMAX / 4 / kThreads : 1;
            V v[NQ][4];
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const uint32_t j = uint32_t(u) * kThreads + tid;
                if (j < E / 4) {
                    const uint32_t i0 = insert0_32(insert0_32(j, llo), lhi);
                    v[u][0] = tile[i0];
                    v[u][1] = tile[i0 + wb];
                    v[u][2] = tile[i0 + wa];
                    v[u][3] = tile[i0 + wa + wb];
                }
            }
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const uint32_t j = uint32_t(u) * kThreads + tid;
                if (j < E / 4) {
                    const uint32_t i0 = insert0_32(insert0_32(j, llo), lhi);
                    V o[4];
                    mv4(G.m, v[u], o);
                    tile[i0] = o[0];
                    tile[i0 + wb] = o[1];
                    tile[i0 + wa] = o[2];
                    tile[i0 + wa + wb] = o[3];
                }
            }
        }
        __syncthreads();
    }

    // ---- store
    {
        V buf[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t e = uint32_t(u) * kThreads + tid;
            if (e < E) buf[u] = tile[e];
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t e = uint32_t(u) * kThreads + tid;
            if (e < E) {
                const uint64_t dm = deposit(uint32_t(u), hdr->pos + 8, k - 8 > 0 ? k - 8 : 0);
                s[dt | dm] = buf[u];
            }
        }
    }
}

template <typename R>
hipError_t run_passes_t(qsv_ctx ctx, void* s, int n, const std::vector<PGate>& gates,
                        const std::vector<Pass>& passes) {
    using V = typename V2T<R>::type;
    constexpr int KMAX = TileK<R>::value;
    // layout of the upload: for each tile pass, a header followed by its gates
    size_t bytes = 0;
    std::vector<size_t> offs(passes.size(), 0);
    for (size_t i = 0; i < passes.size(); ++i) {
        if (passes[i].single) continue;
        offs[i] = bytes;
        bytes += sizeof(TPassHdr) + passes[i].gates.size() * sizeof(TGate<R>);
        bytes = (bytes + 255) & ~size_t(255);
    }
    char* dev = nullptr;
    if (bytes) {
        void* host = nullptr;
        hipError_t e = plan_staging(ctx, bytes, &host);
        if (e != hipSuccess) return e;
        char* h = static_cast<char*>(host);
        for (size_t i = 0; i < passes.size(); ++i) {
            const Pass& ps = passes[i];
            if (ps.single) continue;
            TPassHdr* hd = reinterpret_cast<TPassHdr*>(h + offs[i]);
            hd->k = ps.k;
            hd->ngates = int32_t(ps.gates.size());
            int loc[64];
            for (int p = 0; p < 64; ++p) loc[p] = -1;
            for (int b = 0; b < 24; ++b) hd->pos[b] = b < ps.k ? ps.pos[b] : 0;
            for (int b = 0; b < ps.k; ++b) loc[ps.pos[b]] = b;
            TGate<R>* tg = reinterpret_cast<TGate<R>*>(h + offs[i] + sizeof(TPassHdr));
            for (size_t gi = 0; gi < ps.gates.size(); ++gi) {
                const PGate& g = gates[ps.gates[gi]];
                tg[gi].kind = g.kind;
                tg[gi].l0 = loc[g.p0];
                tg[gi].l1 = g.kind == QSV_G1Q ? 0 : loc[g.p1];
                tg[gi].cs = g.cs;
                for (int m = 0; m < 32; ++m) tg[gi].m[m] = R(g.m[m]);
            }
        }
        void* d = nullptr;
        e = plan_upload(ctx, bytes, &d);
        if (e != hipSuccess) return e;
        dev = static_cast<char*>(d);
    }
    const char* pname = sizeof(R) == 8 ? "tile_pass_c128" : "tile_pass_c64";
    for (size_t i = 0; i < passes.size(); ++i) {
        const Pass& ps = passes[i];
        hipError_t e;
        if (ps.single) {
            e = launch_gate(ctx, s, n, sizeof(R) == 8 ? QSV_C128 : QSV_C64, gates[ps.gates[0]]);
        } else {
            if (n - ps.k > 30) return hipErrorInvalidConfiguration;   // grid limit
            const unsigned tiles = unsigned(uint64_t(1) << (n - ps.k));
            prof_before(ctx, pname, 2.0 * double(uint64_t(1) << n) * sizeof(V));
            hipLaunchKernelGGL((k_tile<R, KMAX>), dim3(tiles), dim3(kThreads), 0, ctx->stream,
                               static_cast<V*>(s), reinterpret_cast<const TPassHdr*>(dev + offs[i]),
                               reinterpret_cast<const TGate<R>*>(dev + offs[i] + sizeof(TPassHdr)));
            prof_after(ctx);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

int tile_bits_max(int dtype) { return dtype == QSV_C128 ? TileK<double>::value : TileK<float>::value; }

hipError_t run_passes(qsv_ctx ctx, void* s, int n, int dtype, const std::vector<PGate>& gates,
                      const std::vector<Pass>& passes) {
    return dtype == QSV_C128 ? run_passes_t<double>(ctx, s, n, gates, passes)
                             : run_passes_t<float>(ctx, s, n, gates, passes);
}

}  // namespace qsv
