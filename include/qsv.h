/*
 * qsv.h -- C ABI of the MI355X (gfx950) state-vector gate engine.
 *
 * The library applies quantum gates to a state vector of 2^n complex
 * amplitudes held in device memory (HBM), following Sec. 2 of "QCLAB++:
 * Simulating Quantum Circuits on GPUs" (arXiv 2303.00123):
 *     psi = (I_l (x) U (x) I_r) phi                                  (eq. 1)
 * for 1-qubit (Sec. 2.1, Alg. 1), controlled 1-qubit (Sec. 2.2, Alg. 2) and
 * 2-qubit gates on any pair of qubits (Sec. 2.3, Alg. 3), plus fused circuits,
 * reductions (norm, Z-string expectations, inner products, single-qubit
 * probabilities and measurement), adjoint-method gradients and batched runs.
 *
 * Conventions (all entry points)
 * ------------------------------
 * - Amplitude order is the paper's big-endian binary representation
 *   (Definition 1, Sec. 2): amplitude index j = sum_i j_i 2^(n-1-i), so qubit
 *   0 is the MOST significant index bit and qubit q has index weight
 *   2^(n-1-q).
 * - Storage: interleaved (re, im) pairs, contiguous, no padding.
 *   QSV_C128: 2 x double per amplitude (16 B); QSV_C64: 2 x float (8 B).
 * - Gate matrices always arrive as host arrays of double in row-major order
 *   of (re, im) pairs; for QSV_C64 states they are rounded once to float.
 *   2x2: 8 doubles.  4x4: 32 doubles, rows/columns indexed by 2*x_qa + x_qb
 *   for a 2-qubit gate on (qa, qb) -- the order eq. (1) gives when qa sits
 *   directly left of qb.  (Alg. 3 as printed pairs its second row with the
 *   higher-weight qubit; eq. (1) decides, and this ABI follows eq. (1).)
 * - Qubit masks (observables) use qubit numbers: bit q set = qubit q.
 * - Ownership: a wrapped buffer belongs to the caller (e.g. a torch tensor)
 *   and is never freed by the library; qsv_state_alloc buffers belong to the
 *   state handle.  A context owns its scratch and staging memory.
 * - Errors: every argument is validated before any work is enqueued, so a
 *   call that returns an error has left the state untouched.  No C++
 *   exception crosses this interface.  qsv_last_error(ctx) gives the text of
 *   the last error on that context.
 * - Asynchrony: gate calls enqueue work on the context's HIP stream and
 *   return immediately.  Calls that return host scalars (norm, expectation,
 *   inner product, probability, measurement, adjoint, batch) synchronise
 *   that stream before returning.
 * - Threading: a context is not thread-safe; use one context per stream.
 */
#ifndef QSV_H_
#define QSV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qsv_status;

enum {
    QSV_OK = 0,
    QSV_ERR_ARG = 1,     /* null pointer, bad count, bad flag, bad control state   */
    QSV_ERR_QUBIT = 2,   /* qubit index out of range or repeated                   */
    QSV_ERR_NOMEM = 3,   /* device or pinned host allocation failed / too large    */
    QSV_ERR_HIP = 4,     /* a HIP runtime call failed (text in qsv_last_error)     */
    QSV_ERR_DTYPE = 5,   /* unknown dtype or mismatched dtypes                     */
    QSV_ERR_ALIGN = 6,   /* device pointer not 16-byte aligned                     */
    QSV_ERR_SIZE = 7,    /* buffer smaller than 2^n amplitudes / n out of range    */
    QSV_ERR_INTERNAL = 8 /* the planner produced an inconsistent plan (a bug)      */
};

enum { QSV_C64 = 1, QSV_C128 = 2 };

/* gate kinds of qsv_gate */
enum {
    QSV_G1Q = 0,    /* 1-qubit gate U (2x2) on q0                                 */
    QSV_GC1Q = 1,   /* U on target q1 where control qubit q0 == ctrl_state        */
    QSV_G2Q = 2,    /* U (4x4, local index 2*x_q0 + x_q1) on (q0, q1)             */
    QSV_GROT = 3    /* exp(-i theta P/2), P = Pauli `axis`, theta = params[param] */
};
enum { QSV_AXIS_X = 0, QSV_AXIS_Y = 1, QSV_AXIS_Z = 2 };

/* flags of qsv_apply_circuit / qsv_adjoint / qsv_batch_run */
enum {
    QSV_FLAG_NO_FUSE = 1,        /* one kernel per gate (Algs. 1-3 unfused)          */
    QSV_FLAG_FORWARD = 2,        /* qsv_adjoint: run the circuit from |0...0> first  */
    QSV_FLAG_CAPTURE_GRAPH = 4,  /* qsv_batch_run: capture and replay a hipGraph     */
    QSV_FLAG_TUNE = 8,           /* qsv_batch_run, qsv_apply_circuit: autotune the tile shape */
    QSV_FLAG_FROM_ZERO = 16      /* qsv_apply_circuit: start from |0...0>, see there  */
};

typedef struct qsv_ctx_s* qsv_ctx;
typedef struct qsv_state_s* qsv_state;

/* One gate of a circuit.  Field use by kind:
 *   QSV_G1Q : q0 = target, m[0..7]
 *   QSV_GC1Q: q0 = control, q1 = target, ctrl_state in {0,1}, m[0..7]
 *   QSV_G2Q : (q0, q1) = (qa, qb), m[0..31]
 *   QSV_GROT: q0 = target, axis, param (index into the params array)
 * Extra controls (Sec. 2.4, Fig. 5), any kind: cmask (bit q = qubit q) names
 * further control qubits, disjoint from the gate's own qubits, and cvals
 * (a subset of cmask) the values they must hold.  The gate then applies
 *     P (x) G + (I - P) (x) I,   P = prod_{q in cmask} |v_q><v_q|_q,
 * i.e. G acts only on the amplitudes whose control bits all hold their
 * values (a Toffoli is X on q0 with two extra controls).  cmask = 0: none.
 * In fused circuits a 1-qubit gate with exactly two controls in all (a
 * QSV_G1Q with two extra controls, or a QSV_GC1Q with one) is rewritten
 * exactly as five controlled 1-qubit gates (V^2 = U, Barenco et al. 1995)
 * and fuses like them; any other gate with extra controls runs as a pass of
 * its own over the amplitudes it changes.  qsv_batch_run and the rotations
 * of qsv_adjoint reject extra controls. */
typedef struct {
    int32_t kind;
    int32_t q0, q1;
    int32_t ctrl_state;
    int32_t axis;
    int32_t param;
    double m[32];
    uint64_t cmask;
    uint64_t cvals;
} qsv_gate;

/* Per-kernel timing collected while profiling is on (see qsv_profile_*). */
typedef struct {
    char name[48];       /* kernel family, e.g. "tile_pass_c128"                 */
    int64_t launches;    /* launches timed                                        */
    double ms;           /* summed HIP-event duration of those launches           */
    double bytes;        /* summed algorithmic HBM bytes of those launches        */
} qsv_kstat;

/* ------------------------------------------------------------------ context */

/* Create a context bound to `hip_stream` (a hipStream_t; NULL = the null
 * stream) on the current HIP device.  *out receives the handle. */
qsv_status qsv_ctx_create(void* hip_stream, qsv_ctx* out);
/* Rebind the context to another stream of the same device. */
qsv_status qsv_ctx_set_stream(qsv_ctx ctx, void* hip_stream);
/* Destroy the context and the memory it owns.  States created on it must be
 * freed first. */
qsv_status qsv_ctx_destroy(qsv_ctx ctx);
/* Wait for all work enqueued on the context's stream. */
qsv_status qsv_sync(qsv_ctx ctx);
/* Static text for a status code; never NULL. */
const char* qsv_status_str(qsv_status s);
/* Text of the last error raised on ctx ("" if none); valid until the next call. */
const char* qsv_last_error(qsv_ctx ctx);

/* -------------------------------------------------------------------- state */

/* Wrap caller-owned device memory as an n-qubit state (Definition 1 order).
 * dev_ptr: device pointer, 16-byte aligned, at least 2^n amplitudes
 * (nbytes >= 2^n * 16 for QSV_C128, 2^n * 8 for QSV_C64).
 * 1 <= n <= 36.  The contents are left as they are. */
qsv_status qsv_state_wrap(qsv_ctx ctx, void* dev_ptr, size_t nbytes, int n, int dtype,
                          qsv_state* out);
/* Allocate an n-qubit state in device memory owned by the handle
 * (uninitialised).  QSV_ERR_NOMEM if the allocation fails. */
qsv_status qsv_state_alloc(qsv_ctx ctx, int n, int dtype, qsv_state* out);
/* Release the handle; frees the buffer only if qsv_state_alloc made it. */
qsv_status qsv_state_free(qsv_state st);
/* Query the handle: any output pointer may be NULL. */
qsv_status qsv_state_info(qsv_state st, int* n, int* dtype, void** dev_ptr);

/* |b>: amplitude b set to 1, every other amplitude to 0 (Definition 1
 * numbering).  b < 2^n. */
qsv_status qsv_init_basis(qsv_state st, uint64_t b);

/* ---------------------------------------------------------------- gates */

/* 1-qubit gate U on qubit q (Sec. 2.1, eq. 1-qubit matvec, Alg. 1): for every
 * pair (a_j, b_j) differing only in qubit q's bit,
 *   psi[a_j] = u00 phi[a_j] + u01 phi[b_j],  psi[b_j] = u10 phi[a_j] + u11 phi[b_j].
 * u: 8 doubles (2x2 row-major (re,im)).  In place.  0 <= q < n. */
qsv_status qsv_apply1q(qsv_state st, int q, const double* u);

/* Controlled 1-qubit gate (Sec. 2.2, Alg. 2): U acts on target qt on the
 * half of the state whose control qubit qc equals ctrl_state (0 or 1); the
 * other half is untouched.  qc != qt, both in [0, n), n >= 2. */
qsv_status qsv_applyC1q(qsv_state st, int qc, int qt, int ctrl_state, const double* u);

/* 2-qubit gate (Sec. 2.3, Alg. 3) on any two distinct qubits (contiguous or
 * not): each quad of indices that differ only in the bits of qa and qb is
 * multiplied by U, whose row/column index is 2*x_qa + x_qb.  u: 32 doubles. */
qsv_status qsv_apply2q(qsv_state st, int qa, int qb, const double* u);

/* Multi-controlled 1-qubit gate (Sec. 2.4, Fig. 5): U acts on target qt on
 * the amplitudes whose controls[i] bits all equal ctrl_states[i] (each 0 or
 * 1; ctrl_states may be NULL for all 1), the rest is untouched.  The pairs
 * it updates come from zero-bit insertion at the nctrl + 1 positions of the
 * controls and the target (Algs. 1-2 generalised), so each control halves
 * the amplitudes read and written.  0 <= nctrl <= n - 1, qubits distinct and
 * in [0, n).  u: 8 doubles. */
qsv_status qsv_applyMC1q(qsv_state st, int nctrl, const int* controls, const int* ctrl_states,
                         int qt, const double* u);

/* General k-qubit gate on any k distinct qubits, contiguous or not (Sec.
 * 2.4: the masks of Algs. 1-3 extended by one inserted zero bit per extra
 * qubit).  U is 2^k x 2^k, row-major (re, im) pairs (2 * 4^k doubles),
 * rows/columns indexed by sum_i x_{qubits[i]} 2^(k-1-i): qubits[0] is the
 * most significant bit of the local index, which is eq. (1)'s order when
 * the qubits are contiguous and ascending.  1 <= k <= 5, k <= n.  The matrix
 * is copied to device memory before the call returns.  For k >= 3 the
 * context's matrix-core setting (qsv_set_matrix_cores) picks the kernel. */
qsv_status qsv_applyKq(qsv_state st, int k, const int* qubits, const double* u);

/* Apply gates g[0..ng) in order.  Rotations read params[0..nparams).  By
 * default gates are grouped into fused passes: each pass loads a tile of
 * amplitudes over a set of qubits once from HBM, applies every gate of the
 * group to it, and stores it once.  Gates on disjoint qubits are reordered
 * only where they commute.  QSV_FLAG_NO_FUSE applies one kernel per gate.
 * QSV_FLAG_FROM_ZERO: the state is first set to |0...0>, as qsv_init_basis
 * with b = 0 would, and the result is the circuit applied to that; when the
 * first pass is a fused one it makes |0...0> in registers instead of reading
 * the state, which saves one write and one read of it.
 * QSV_FLAG_TUNE (with QSV_FLAG_FROM_ZERO only): on the first call for a
 * circuit structure (qubit count, precision, kernel mode, gate kinds, qubits
 * and controls) run the circuit from |0...0> twice with each candidate tile
 * shape -- (tile_bits, reg_bits, exchange) = (13, 5, split), (12, 4, split),
 * (12, 4, full), (12, 3, split), (11, 3, split) -- and keep the shape of the
 * fastest second run for later calls with the flag on this context; the
 * state ends as the circuit's result either way.  With specialised kernels
 * (qsv_set_jit) the tuning call also compiles every candidate shape's pass
 * kernels.  Calls without the flag use the context's tile shape
 * (qsv_set_tile). */
qsv_status qsv_apply_circuit(qsv_state st, const qsv_gate* g, int64_t ng, const double* params,
                             int64_t nparams, int flags);

/* ----------------------------------------------------------- reductions */
/* All reductions accumulate in FP64 (for both dtypes) with a fixed-order
 * two-stage tree, so repeated calls give bit-identical results. */

/* sum_x |psi_x|^2 */
qsv_status qsv_norm2(qsv_state st, double* out);

/* For k < nterms: out_terms[k] = <psi| Z^{qmasks[k]} |psi> where Z^{m} is the
 * product of Pauli Z over the qubits set in m (diagonal, value
 * (-1)^{popcount of the selected bits}).  out_sum = sum_k w[k] out_terms[k].
 * w may be NULL (weights 1); out_terms or out_sum may be NULL.
 * 1 <= nterms <= 4096. */
qsv_status qsv_expect_z(qsv_state st, int nterms, const uint64_t* qmasks, const double* w,
                        double* out_terms, double* out_sum);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * per-term values of qsv_expect_z, out_dev[k] = <psi| Z^{qmasks[k]} |psi>
 * for k < nterms, written to out_dev, a caller-owned device array of at
 * least nterms doubles (8-byte aligned).  Same kernels and summation order
 * as qsv_expect_z, so the values are bit-identical to its out_terms.  The
 * call allocates nothing and does not synchronise: it enqueues kernels on
 * the context's stream and returns (no memset, no copy, so it may be
 * captured into a hipGraph).  qmasks is read on the host before the call
 * returns.  Scratch: a fixed array of 256 KiB + 128 B per GPU, held until
 * the process ends and shared by every call on that GPU (from any context);
 * each call overwrites all of it that it reads, so nothing needs clearing,
 * but calls that overlap in time on one GPU (different streams or threads)
 * race on it and must be ordered by the caller.  1 <= nterms <= 4096. */
qsv_status qsv_expect_z_dev(qsv_state st, int nterms, const uint64_t* qmasks, double* out_dev);

/* <a|b> = sum_x conj(a_x) b_x (out[0] = re, out[1] = im).  a and b must have
 * the same n; their dtypes may differ (the c64 operand is widened). */
qsv_status qsv_inner(qsv_state a, qsv_state b, double* out);

/* Probability that qubit q reads 1: sum over x with bit q set of |psi_x|^2. */
qsv_status qsv_prob1(qsv_state st, int q, double* p1);

/* Projective measurement of qubit q with a caller-supplied uniform draw r in
 * [0,1): outcome 0 iff r < P(q = 0) (both in FP64); the state is projected
 * onto the outcome and renormalised.  *outcome receives 0 or 1. */
qsv_status qsv_measure1(qsv_state st, int q, double r, int* outcome);

/* Host <-> device copies of the whole state (nbytes >= 2^n amplitudes). */
qsv_status qsv_copy_to_host(qsv_state st, void* host, size_t nbytes);
qsv_status qsv_copy_from_host(qsv_state st, const void* host, size_t nbytes);

/* ------------------------------------------------------------- gradients */

/* Adjoint-method gradient (Jones & Gacon, arXiv:2009.02823) of
 *   f(params) = <psi| O |psi>,  psi = U_ng..U_1 |0..0>,  O = sum_k w_k Z^{qmasks[k]}.
 * psi: with QSV_FLAG_FORWARD it is set to |0..0> and the circuit is run;
 *      otherwise it must already hold U|0..0>.  It is consumed: on return it
 *      holds the state rewound through every gate (|0..0> up to rounding).
 * lam: a second state of the same n and dtype, used as the co-state; its
 *      contents on entry are ignored and on return are undefined.
 * Only QSV_GROT gates carry parameters; grad[j] (j < nparams) receives
 * df/dparams[j], summed over every rotation that uses parameter j; *expval
 * receives f.  Every other gate must be unitary (its adjoint is used to
 * rewind).  Both vectors are rewound together, with the partial
 * Im<lam| P |psi> of each rotation fused into its rewind pass. */
qsv_status qsv_adjoint(qsv_state psi, qsv_state lam, const qsv_gate* g, int64_t ng,
                       const double* params, int64_t nparams, int nterms, const uint64_t* qmasks,
                       const double* w, double* expval, double* grad, int flags);

/* ----------------------------------------------------------------- batch */

/* Run nb independent circuits in one persistent launch (for nb >= 32 two
 * launches, one after the other on the same stream, each over half the
 * circuits: the second half is planned and staged on the host while the
 * first one runs).  Circuit b has
 * nq[b] qubits (1 <= nq[b] <= 24), gates g[gate_off[b] .. gate_off[b+1]),
 * rotation angles from params (indices global to the batch), starts in
 * |0..0> and yields out[b] = sum over terms t in [term_off[b], term_off[b+1])
 * of w[t] <Z^{qmasks[t]}> (qubit masks relative to circuit b; w may be NULL
 * for weights 1).  gate_off and term_off have nb + 1 entries starting at 0.
 * dtype selects the state precision (accumulation is FP64 either way).  Each
 * circuit is applied with the fused tile passes of qsv_apply_circuit; the
 * library keeps the multi-pass states in its own device memory, and states
 * of one tile never leave the workgroup.
 * QSV_FLAG_TUNE: on the first call for a batch shape (qubit counts, gate
 * kinds and qubits, observable terms -- not the angles) time each candidate
 * tile shape (best of two runs of the whole batch in one launch) and keep
 * the fastest for later calls (file cache if the environment variable
 * QSV_TUNE_CACHE names one).
 * QSV_FLAG_CAPTURE_GRAPH: capture upload, counter reset, kernel and result
 * download in a hipGraph (one per launch) on a library-owned stream, and
 * replay it on later calls with the same batch shape (new angles are
 * uploaded by the replay).
 * Synchronises before returning.
 * Errors: a workgroup that waits for the previous pass of its circuit gives
 * up after a bounded number of sleeps (about 2 s; the environment variable
 * QSV_BATCH_SPIN_LIMIT, read at each launch or capture, sets the count), the
 * rest of the launch drains without computing, and the call returns
 * QSV_ERR_HIP with "spin limit" in qsv_last_error; out is then not written. */
qsv_status qsv_batch_run(qsv_ctx ctx, int nb, const int* nq, const int64_t* gate_off,
                         const qsv_gate* g, const double* params, int64_t nparams,
                         const int64_t* term_off, const uint64_t* qmasks, const double* w,
                         int dtype, double* out, int flags);

/* -------------------------------------------------------------- profiling */

/* Start timing every kernel the library launches on ctx with HIP events
 * recorded on the context's stream (previous records are discarded). */
qsv_status qsv_profile_begin(qsv_ctx ctx);
/* Stop timing, wait for the stream, and report per-kernel-family totals:
 * up to `max` entries written to out, *count receives the number of
 * families. */
qsv_status qsv_profile_end(qsv_ctx ctx, qsv_kstat* out, int max, int* count);

/* Tile shape of the context's later fused passes for one dtype.
 * tile_bits: log2 of the amplitudes per tile, in [10, 13] (0 = the default, 13).
 * low_bits: number of lowest index bits every tile keeps, so each tile is
 * made of contiguous runs of 2^low_bits amplitudes; in [0, tile_bits - 2]
 * (0 = 3 for QSV_C128, 4 for QSV_C64, i.e. 128-byte runs).
 * reg_bits: log2 of the amplitudes each thread keeps in registers (a tile
 * has 2^(tile_bits - reg_bits) threads; 0 = 5 for tiles of 2^13, 4 for
 * 2^12, else tile_bits - 8).  Compiled (tile_bits, reg_bits) shapes: (10, 2),
 * (11, 3), (12, 3), (12, 4), (13, 4), (13, 5); others give QSV_ERR_ARG.
 * lds_rounds: how a tile changes register mapping between stages: 1 = the
 * whole tile goes through LDS at once; 2 = consecutive stages share a
 * register bit and the tile moves in two halves, so a workgroup needs half
 * the LDS and more workgroups fit on a compute unit (0 = 2).
 * States with fewer than 10 qubits run one kernel per gate.  A launch covers
 * fewer than 2^32 work-items, so a state of more than tile_bits + 23 qubits
 * takes tiles of 2^(n - 23) amplitudes (at most 2^13) regardless. */
qsv_status qsv_set_tile(qsv_ctx ctx, int dtype, int tile_bits, int low_bits, int reg_bits,
                        int lds_rounds);

/* Specialised tile-pass kernels.  mode 1: each fused pass of
 * qsv_apply_circuit on this context runs a kernel generated for that pass's
 * structure (gate kinds and register bits, stage mappings, LDS and global
 * offsets as constants; the matrices are still read from device memory), so
 * each gate is a direct call of its register body, updated in place, instead
 * of an interpreted opcode.  The first run of a new structure compiles its
 * passes with the ROCm device compiler in child processes (several at once;
 * seconds per pass) and keeps them on the context; circuits with the same
 * structure and other angles reuse them.  A pass whose kernel cannot be
 * built (or would spill) runs the interpreting kernel.  mode 0 (the
 * default; the environment variable QSV_JIT=1 sets 1 at context creation):
 * the interpreting kernel only.  QSV_ERR_ARG if mode is 1 and no compiler is
 * found (QSV_JIT_CLANG, else $ROCM_PATH/llvm/bin/clang++, else
 * /opt/rocm/llvm/bin/clang++).  If the environment variable QSV_JIT_CACHE
 * names a directory, accepted kernels are also written there and later
 * processes load them instead of compiling. */
qsv_status qsv_set_jit(qsv_ctx ctx, int mode);
/* Matrix cores for dense k-qubit gates (qsv_applyKq with n - k >= 6): U
 * is applied as real matrix products on the MFMA units, FP64 MFMA for
 * complex128 and FP32 MFMA for complex64 (full precision; only the
 * summation order differs from the vector kernel), 16 groups of 2^k
 * amplitudes per wave.  mode 1 (the default): for k = 3 and 5, where they
 * measured faster than the vector units; mode 2: for every k in 3..5; mode
 * 0: never (the vector kernel, one output row at a time).  Other gates and
 * the fused passes are not affected.  QSV_ERR_ARG for another mode. */
qsv_status qsv_set_matrix_cores(qsv_ctx ctx, int mode);
/* Kernels built or loaded so far on ctx and the wall time spent on it. */
qsv_status qsv_jit_stats(qsv_ctx ctx, int* kernels, double* compile_seconds);
/* Host-only: the generated source of fused pass `pass` of an n-qubit
 * circuit (n >= 10) planned with the default tile shape for dtype (no device
 * work).  *len receives its length; buf (cap bytes, may be NULL) receives it
 * NUL-terminated, else QSV_ERR_SIZE.  QSV_ERR_ARG if the pass is a single
 * gate or out of range. */
qsv_status qsv_jit_source(int n, int dtype, const qsv_gate* g, int64_t ng, const double* params,
                          int64_t nparams, int64_t pass, char* buf, size_t cap, size_t* len);

/* Host-only query of the exact gate sequence the tile kernels would apply for
 * qsv_apply_circuit (no device work; needs no GPU): gates grouped into passes
 * and register stages, with the 1-qubit gates of a stage multiplied into the
 * neighbouring 2-qubit gates.  Tile shape arguments as in qsv_set_tile.  The
 * device records of every pass are built too (and discarded), so a planner
 * inconsistency surfaces here as QSV_ERR_INTERNAL.  out receives up to `cap`
 * records in execution order (kind QSV_G1Q, QSV_GC1Q or QSV_G2Q with explicit
 * matrices; rotations are evaluated with params), pass_of_out[i] the pass of
 * record i (either output may be NULL); *nout receives the number of
 * records, or the number needed if cap is too small (then QSV_ERR_SIZE). */
qsv_status qsv_plan_fused(int n, int dtype, const qsv_gate* g, int64_t ng, const double* params,
                          int64_t nparams, int tile_bits, int low_bits, int reg_bits, int lds_rounds,
                          qsv_gate* out, int64_t cap, int32_t* pass_of_out, int64_t* nout);

/* Host-only query of how the pass planner groups the gates of an n-qubit
 * circuit, taken one to one as given (no device work; needs no GPU), so that
 * every input gate gets a pass.  qsv_apply_circuit first merges neighbouring
 * gates by its cost-aware fusion and plans the merged list, which can need
 * fewer passes; qsv_plan_fused returns exactly what it runs.  tile_bits /
 * low_bits as in qsv_set_tile (0 = defaults for dtype).  Outputs, each an array of at least
 * ng entries: pass_of_gate[i] = pass that applies gate i; exec_order = gate
 * indices in the order the kernels apply them (passes in sequence; inside a
 * pass, its register stages in sequence); pass_qubits[p] = qubit mask (bit q = qubit q)
 * of pass p's tile.  *npasses receives the number of passes. */
qsv_status qsv_plan_circuit(int n, int dtype, const qsv_gate* g, int64_t ng, int tile_bits,
                            int low_bits, int reg_bits, int64_t* npasses, int32_t* pass_of_gate,
                            int32_t* exec_order, uint64_t* pass_qubits);

#ifdef __cplusplus
}
#endif
#endif /* QSV_H_ */
