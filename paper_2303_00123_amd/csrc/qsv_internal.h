// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "qsv.h"

namespace qsv {

constexpr int kMaxQubits = 36;
constexpr int kMaxTileBits = 13;       // largest compiled tile (2^13 amplitudes)
constexpr int kMaxTileGridLog2 = 23;   // tiles per launch (256 threads each, < 2^32 work-items)

inline size_t amp_bytes(int dtype) { return dtype == QSV_C128 ? 16 : 8; }

// ---------------------------------------------------------------- plans
// A gate in index-bit coordinates: position p = n-1-q of qubit q.
struct PGate {
    int kind;       // QSV_G1Q, QSV_GC1Q, QSV_G2Q (rotations are lowered to G1Q), or KROT
    int p0, p1;     // G1Q: p0 target; GC1Q: p0 control, p1 target; G2Q: p0 = pos(qa), p1 = pos(qb)
    int cs;
    double m[32];
    int tag = -1;   // adjoint sweep: index of the forward gate a KROT rewinds
    // extra controls (Sec. 2.4) as index-bit masks: the gate acts where the
    // bits in cm equal those of cv.  Such a gate is never fused: it runs as
    // its own pass (k_mc) and orders every gate around it.
    uint64_t cm = 0, cv = 0;
};

// Internal kind for the adjoint sweep: a rotation exp(-i theta P/2) being
// rewound.  p0 = target, cs = Pauli axis, p1 = its partial-sum slot in the
// pass, m = the 2x2 U^dagger.  Never fused with other gates.
constexpr int KROT = 16;
inline bool is_1q(int kind) { return kind == QSV_G1Q || kind == KROT; }

inline int coal_bits_for(int dtype) { return dtype == QSV_C128 ? 3 : 4; }

// A stage of a tile pass: the gates applied while each thread holds the
// amplitudes spanning `rbits` (local tile bits) in registers.
struct Stage {
    int nr = 0;                  // register bits of the pass's kernel
    int rbits[8] = {0};          // register bit j <-> local tile bit rbits[j]
    int hprev = -1;              // split exchange: local bit shared with the previous stage
                                 // (it is rbits[nr - 1]); -1 for the first stage
    std::vector<int> gates;      // indices into the lowered gate list, in execution order
};

// One fused pass over the state.
struct Pass {
    bool single = false;         // true: one gate, unfused kernel
    int k = 0;                   // tile bits (tile = 2^k amplitudes)
    int rb = 0;                  // register bits per thread (2^(k - rb) threads)
    int coal = 0;                // local bits the first/last stage keep on lanes
    bool split = false;          // stage changes go through half the tile in LDS, in two
                                 // rounds split on a register bit shared by both stages
    int pos[24] = {0};           // ascending global bit positions of the tile's local bits
    std::vector<int> gates;      // indices into the lowered gate list, in execution order
    std::vector<Stage> stages;   // stage 0 and the last stage use the canonical mapping
};

struct TileConfig {
    int tile_bits;   // log2 amplitudes per tile
    int low_bits;    // contiguous low bits kept in every tile
    int reg_bits;    // log2 amplitudes per thread (threads per tile = 2^(tile_bits - reg_bits))
    int coal_bits;   // the first and last stage keep local bits [0, coal_bits) on lanes, so
                     // global loads and stores move 2^coal_bits contiguous amplitudes per lane group
    int split = 0;   // 1: split stage changes (half the tile in LDS, see Pass::split)
};

constexpr int kTileThreads = 256;   // threads per workgroup of the batch and adjoint kernels
constexpr int kMinTileBits = 10;    // at least 2 register bits per thread
constexpr int kDefaultTileBits = 13;   // 2^13 amplitudes, 32 per thread, split LDS exchange
constexpr int kDefaultRegBits = 5;

// (tile_bits, reg_bits) pairs the single-state tile kernel is compiled for
bool tile_shape_supported(int dtype, int tile_bits, int reg_bits);

// Group gates into passes (greedy, dependency-respecting), then split each
// tile pass into register stages.
std::vector<Pass> plan_passes(int n, const std::vector<PGate>& gates, const TileConfig& cfg);
// Register stages of one pass whose k, rb, coal, split, pos and gates are set.
void plan_pass_stages(int n, const std::vector<PGate>& gates, Pass& ps);

// Fuse the gates of one register stage (indices into `gates`, in execution
// order): 1-qubit gates are multiplied into the next 2-qubit or controlled
// gate on the same qubit (or emitted at the end of the stage), and a 2-qubit
// gate directly following another on the same pair is merged into it.  The
// result applies the same operator with fewer kernel dispatches.
std::vector<PGate> fuse_stage(const std::vector<PGate>& gates, const std::vector<int>& idx);

// The same fusion over a whole circuit, applied before pass planning when the
// state is large enough for tile passes (below that, gates run one by one).
// 1-qubit gates with exactly two controls are first rewritten exactly as
// two-qubit gates (expand_double_controls) so that they fuse too.
std::vector<PGate> prefuse(const std::vector<PGate>& gates);
std::vector<PGate> expand_double_controls(const std::vector<PGate>& gates);
// A unitary square root of a 2x2 unitary (row-major (re, im) pairs).
void unitary_sqrt2(const double* u, double* r);

// Device-side gate kinds inside a tile pass.
enum {
    DK_1Q = 0,    // generic 2x2 on register bit r0
    DK_1D = 1,    // diagonal 2x2: m[0..1] = d0, m[2..3] = d1
    DK_C1Q = 2,   // generic 2x2 on r1 where register bit r0 == cs
    DK_CX = 3,    // swap on r1 where r0 == cs (controlled X)
    DK_CD = 4,    // diagonal (d0, d1) on r1 where r0 == cs
    DK_2Q = 5,    // generic 4x4 on (r0, r1), local index 2*x_r0 + x_r1
    DK_ROT = 6,   // adjoint sweep: partial Im<lam|P|psi> into slot r1, then 2x2 m on r0; P = axis cs
    DK_1R = 8     // real 2x2 on register bit r0 (m[0], m[2], m[4], m[6]; imaginary parts zero)
};

// Device-side gate record of a tile pass (register bit coordinates).
template <typename R>
struct TGate {
    int32_t kind;
    int32_t r0, r1;
    int32_t cs;
    R m[32];
};

// Stage record in device memory.
struct TStage {
    int32_t gbeg, gend;     // gate range [gbeg, gend) of the pass's gate array
    int32_t tbits[10];      // thread-id bit j <-> local bit
    uint32_t su[32];        // byte offset (after the LDS swizzle) of register slot u (reads)
    uint32_t su_wr[32];     // the same for the write at the stage's end: su of the slot the
                            // amplitude belongs to after the stage's trailing permutation gates
    // split exchange (half the tile in LDS): the bit shared with the previous
    // stage is removed from the read addresses, the one shared with the next
    // stage from the write addresses (su and su_wr are then half-tile offsets)
    int32_t jw;             // register index of the bit shared with the next stage (-1: none)
    int32_t tbr[10];        // thread bit j -> half-tile address bit, reads
    int32_t tbw[10];        // thread bit j -> half-tile address bit, writes
};

// Pass header in device memory; followed by nstages TStage records and then
// the pass's TGate records.
struct TPassHdr {
    int32_t k;
    int32_t nstages;
    int32_t ngates;
    int32_t pad;            // adjoint passes: number of rotation partial-sum slots
    int32_t rb;             // register bits
    int32_t pad2;
    int32_t pos[24];
    int32_t tpos_ld[10];    // global position of thread-id bit j in the load mapping
    int32_t tpos_st[10];    // ... in the store mapping
    uint64_t du[32];        // amplitude offset of register slot u in the load mapping
    uint64_t du_st[32];     // ... in the store mapping
};

// LDS slot swizzle of the tile kernels: an XOR of the slot index with a fold
// of its higher bits into the bank-selecting low bits.  It is linear over
// GF(2), so swz(a | b) = swz(a) ^ swz(b) for disjoint a, b.
__host__ __device__ inline uint32_t tile_swz(uint32_t e, int elem_bytes) {
    return elem_bytes == 16 ? e ^ (((e >> 4) ^ (e >> 8) ^ (e >> 12)) & 15u)
                            : e ^ (((e >> 5) ^ (e >> 10)) & 31u);
}

// ------------------------------------------------------------- profiling
struct ProfRec {
    const char* name;
    double bytes;
    hipEvent_t start, stop;
};

// Pass plan of the last circuit planned through it, keyed by what planning
// depends on: the qubit count, the tile shape and the positions and kinds of
// the fused gates (not their matrices).  A circuit evaluated again with new
// angles keeps its plan; only the device records are rewritten.
struct PlanMemo {
    int n = -1;
    TileConfig cfg{0, 0, 0, 0};
    std::vector<uint32_t> sig;
    std::vector<Pass> passes;
};
}  // namespace qsv

namespace qsv {
// Buffers of one part of a batch call: device [upload | counters | out |
// partials | states], pinned staging and results, the captured graph and
// the per-circuit plan memo.
struct BatchSlot {
    void* d = nullptr;
    size_t d_bytes = 0;
    void* h = nullptr;
    size_t h_bytes = 0;
    double* h_out = nullptr;
    size_t h_out_n = 0;
    size_t ctr_off = 0, out_off = 0, part_off = 0, state_off = 0;
    void* graph_exec = nullptr;   // hipGraphExec_t
    uint64_t graph_key = 0;
    std::vector<PlanMemo> memo;
};

// Host worker threads that run f(arg, i) for i in [0, n) together with the
// calling thread (qsv_pool.cpp).  pool_run returns false if a call threw;
// one caller at a time per pool.
class WorkerPool;
WorkerPool* pool_create(int workers);   // nullptr if no thread could be started
void pool_destroy(WorkerPool* p);
bool pool_run(WorkerPool* p, int n, void (*f)(void*, int), void* arg);

// A specialised tile-pass kernel (qsv_jit.cpp); fn null = not available for
// that pass structure (the interpreting kernel runs it).
struct JitKernel {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
};
}  // namespace qsv

struct qsv_ctx_s {
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cus = 256;
    std::string last_error;

    // reduction scratch: stage-1 partials and stage-2 results (fixed size)
    double* d_red = nullptr;
    double* h_red = nullptr;     // pinned, receives stage-2 results
    // plan upload: pinned staging + device copy (grown on demand)
    void* d_plan = nullptr;
    size_t d_plan_bytes = 0;
    void* h_plan = nullptr;
    size_t h_plan_bytes = 0;
    hipEvent_t plan_copied = nullptr;   // last H2D plan copy done -> h_plan reusable
    // auxiliary device buffer (grown on demand): adjoint per-gate gradients
    double* d_aux = nullptr;
    size_t d_aux_doubles = 0;

    qsv::TileConfig tile_c128{13, 3, 5, 3, 1};
    qsv::TileConfig tile_c64{13, 4, 5, 4, 1};

    // profiling
    bool profiling = false;
    std::vector<qsv::ProfRec> prof;
    std::vector<hipEvent_t> event_pool;
    size_t event_next = 0;

    // batch: a call runs in up to two parts (qsv_batch.hip), each with its
    // own buffers, plan memo and captured graph
    qsv::BatchSlot batch[2];
    hipStream_t batch_stream = nullptr;   // capture stream (default priority)

    // autotuner choices: batch shape key -> (tile_bits, low_bits)
    std::map<uint64_t, std::pair<int, int>> tuned;
    bool tune_loaded = false;

    // plan of the last fused circuit: reused while the lowered gates, the
    // qubit count, the precision and the tile shape are unchanged
    std::vector<qsv::PGate> cache_in;   // lowered gates the plan was made from
    int cache_n = -1;
    int cache_dtype = 0;
    qsv::TileConfig cache_cfg{0, 0, 0, 0};
    std::vector<qsv::PGate> cache_pg;   // fused gates
    qsv::PlanMemo memo;                 // their passes
    bool plan_resident = false;         // d_plan holds the records of memo.passes
    qsv::PlanMemo adj_memo;             // passes of the last adjoint sweep's reversed circuit

    // single-state tuner (QSV_FLAG_TUNE on qsv_apply_circuit): circuit
    // structure key -> chosen tile shape
    std::map<uint64_t, qsv::TileConfig> tuned_single;

    // dense k-qubit gates on the matrix cores (qsv_set_matrix_cores)
    int kq_mfma = 1;

    // host worker threads of the batch planner (started on first use)
    qsv::WorkerPool* pool = nullptr;

    // specialised tile-pass kernels (qsv_set_jit): by record-structure hash,
    // and those of the resident plan (valid while plan_resident)
    int jit_mode = 0;
    std::map<uint64_t, qsv::JitKernel> jit_kernels;
    std::vector<hipFunction_t> jit_plan_fns;
    double jit_compile_s = 0.0;
    int jit_compiled = 0;
};

struct qsv_state_s {
    qsv_ctx ctx = nullptr;
    void* ptr = nullptr;
    int n = 0;
    int dtype = QSV_C128;
    bool owns = false;
    size_t nbytes = 0;
};

namespace qsv {

constexpr size_t kRedDoubles = 1 << 16;   // partials: up to 2048 blocks x 16 terms, + results

// Plan upload (capi.cpp): returns a pinned host buffer of at least `bytes`
// that is safe to overwrite, and after filling it, copies it to device memory.
hipError_t plan_staging(qsv_ctx ctx, size_t bytes, void** host);
hipError_t plan_upload(qsv_ctx ctx, size_t bytes, void** dev);
hipError_t ensure_aux(qsv_ctx ctx, size_t doubles);

// profiling helpers: bracket a launch (on the context stream, or on `stream`)
void prof_before(qsv_ctx ctx, const char* name, double bytes);
void prof_after(qsv_ctx ctx);
void prof_before_on(qsv_ctx ctx, hipStream_t stream, const char* name, double bytes);
void prof_after_on(qsv_ctx ctx, hipStream_t stream);

// Diagnostics to stderr when the environment variable QSV_LOG is set to a
// non-zero value (planner decisions, launch shapes, host planning time).
bool log_enabled();
void logf(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// exp(-i theta P / 2) for Pauli `axis`, as a 2x2 row-major (re, im) matrix
void rotation_matrix(int axis, double theta, double* m);

constexpr int kMaxBatchQubits = 24;

// Autotuner cache (qsv_tune.cpp): tuned tile shape for a batch shape key,
// kept per context and, if QSV_TUNE_CACHE names a file, across processes.
bool tune_lookup(qsv_ctx ctx, uint64_t key, int dtype, int* tile_bits, int* low_bits);
void tune_store(qsv_ctx ctx, uint64_t key, int dtype, int tile_bits, int low_bits, double ms);

// ------------------------------------------------------------ launchers
// All launchers enqueue on ctx->stream and return the launch status.
hipError_t launch_init_basis(qsv_ctx ctx, void* s, int n, int dtype, uint64_t b);
hipError_t launch_apply1q(qsv_ctx ctx, void* s, int n, int dtype, int p, const double* u);
hipError_t launch_applyc1q(qsv_ctx ctx, void* s, int n, int dtype, int pc, int pt, int cs,
                           const double* u);
hipError_t launch_apply2q(qsv_ctx ctx, void* s, int n, int dtype, int pa, int pb, const double* u);
hipError_t launch_gate(qsv_ctx ctx, void* s, int n, int dtype, const PGate& g);
// k-qubit gate (1 <= k <= 5) on index-bit positions pos[0..k) (pos[0] = most
// significant local bit); du: the 2^k x 2^k matrix in device memory, in the
// state's real type.
hipError_t launch_kq(qsv_ctx ctx, void* s, int n, int dtype, int k, const int* pos, const void* du,
                     bool mfma = false);
// the matrix-core form of the k-qubit gate applies at this size and
// qsv_set_matrix_cores mode; its matrix is 4^(k+1) reals in the lane order
// kq_mfma_pack writes (u as for qsv_applyKq)
bool kq_mfma_applies(int n, int k, int mode);
void kq_mfma_pack(int dtype, int k, const double* u, void* out);

// Largest tile (log2 amplitudes) the tile kernel supports for a dtype.
int tile_bits_max(int dtype);

// Device record of one tile pass (header, stages, fused gates): its size
// bound and its contents (false on a planner inconsistency).
size_t pass_record_bytes(int dtype, const Pass& ps);
bool write_pass_record(int dtype, char* dst, const std::vector<PGate>& gates, const Pass& ps);

const std::vector<Pass>& plan_memo(PlanMemo& m, int n, const std::vector<PGate>& fused, const TileConfig& cfg);

// Tile passes: uploads the plan for all passes, then launches them in order.
// cached: the passes are ctx->memo.passes; their records are uploaded only
// if d_plan no longer holds them.
hipError_t run_passes(qsv_ctx ctx, void* s, int n, int dtype, const std::vector<PGate>& gates,
                      const std::vector<Pass>& passes, bool cached = false, bool from_zero = false);

// Specialised tile-pass kernels (qsv_jit.cpp).  jit_prepare makes sure each
// host record in recs (null entries are skipped) has a kernel; fns[i] is
// null where none could be built.
bool jit_available();
uint64_t jit_record_key(int dtype, const char* rec, bool split);
std::string jit_pass_source(int dtype, const char* rec, bool split, const std::string& fname);
hipError_t jit_prepare(qsv_ctx ctx, int dtype, const std::vector<const char*>& recs,
                       const std::vector<bool>& split, std::vector<hipFunction_t>& fns);
void jit_release(qsv_ctx ctx);

// Reductions.  Stage-1 partials go to ctx scratch; results land in host memory.
// Z-string sums: out[t] = sum_x |s_x|^2 (-1)^{popcount(x & pmask[t])}, t < nt.
hipError_t reduce_zstrings(qsv_ctx ctx, const void* s, int n, int dtype, int nt,
                           const uint64_t* pmasks, double* out);
// The same sums for qubit masks qmasks[0..nt) (bit q = qubit q), written to
// out_dev (device memory) with no allocation and no host synchronisation;
// partials live in a fixed per-GPU array whose address reduce_scratch_init
// (called once per device, with that device current) looks up.
hipError_t reduce_scratch_init(int device);
hipError_t reduce_zstrings_dev(qsv_ctx ctx, const void* s, int n, int dtype, int nt,
                               const uint64_t* qmasks, double* out_dev);
// out[0] = sum over x with bit p clear, out[1] = with bit p set, of |s_x|^2.
hipError_t reduce_bit_split(qsv_ctx ctx, const void* s, int n, int dtype, int p, double* out);
// <a|b>
hipError_t reduce_inner(qsv_ctx ctx, const void* a, int dta, const void* b, int dtb, int n,
                        double* out);
// keep amplitudes whose bit p equals `keep`, scaled by `scale`; zero the rest.
hipError_t launch_collapse(qsv_ctx ctx, void* s, int n, int dtype, int p, int keep, double scale);

// Adjoint sweep (qsv_adjoint.hip).  fused: rewind through two-vector tile
// passes; otherwise one kernel per gate.
hipError_t run_adjoint(qsv_ctx ctx, void* psi, void* lam, int n, int dtype,
                       const std::vector<PGate>& fwd, const std::vector<int>& rot_param,
                       const std::vector<int>& rot_axis, int nterms, const uint64_t* pmasks,
                       const double* w, double* grad_by_gate, bool fused);

}  // namespace qsv
