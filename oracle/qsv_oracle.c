/*
 * FP64 CPU oracle for state-vector gate application.  TEST INFRASTRUCTURE
 * ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg use
 * it; the GPU library never links, loads or calls it, and it shares no code
 * with it.
 *
 * Every gate is applied by its plain definition, eq. (1) of Sec. 2:
 *     psi = (I_l (x) U (x) I_r) phi,
 * evaluated entry by entry: psi[x] = sum_y M[x,y] phi[y], where the Kronecker
 * structure makes M[x,y] = U[row(x), col(y)] when x and y agree on every
 * qubit the gate does not touch, and 0 otherwise.  Rows and columns of U are
 * the gate qubits' bits read with Definition 1 (big-endian: qubit 0 is the
 * most significant bit of x).  A controlled gate (Sec. 2.2) is
 *     |not cs><not cs|_qc (x) I  +  |cs><cs|_qc (x) U_qt.
 * All applications are out of place (phi -> psi); nothing here uses the
 * zero-bit-insertion index maps of Algs. 1-3.
 *
 * Readings where the paper is silent (listed with the other readings of the
 * paper in the design notes):
 *  - 2-qubit local basis: row/col index 2*x_qa + x_qb for the gate's qubits
 *    (qa, qb) in the order given, i.e. eq. (1) for qa directly left of qb.
 *  - Rotations: R_P(theta) = exp(-i theta P / 2) = cos(theta/2) I
 *    - i sin(theta/2) P for P in {X, Y, Z}.
 *  - Gradients follow the adjoint method of Jones & Gacon (arXiv:2009.02823),
 *    the parameter-shift rule (exact for exp(-i theta P / 2)) and central
 *    finite differences.
 *
 * Sums over the state use Neumaier-compensated summation, so the reference
 * reductions carry ~1 ulp of error independent of 2^n.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double ORC_PI = 3.14159265358979323846;

/* gate kinds understood by the oracle (the Python marshaller fills these) */
enum { ORC_1Q = 0, ORC_C1Q = 1, ORC_2Q = 2, ORC_ROT = 3 };

typedef struct {
    int32_t kind;
    int32_t q0, q1;      /* 1q/rot: q0 target; c1q: q0 control, q1 target; 2q: (qa, qb) */
    int32_t ctrl_state;  /* c1q */
    int32_t axis;        /* rot: 0 = X, 1 = Y, 2 = Z */
    int32_t param;       /* rot: index into params */
    double m[32];        /* row-major (re, im) pairs: 2x2 uses 8, 4x4 uses 32 */
    uint64_t cmask;      /* extra control qubits (bit q = qubit q), 0 = none    */
    uint64_t cvals;      /* the values they must hold (bit q), within cmask     */
} orc_gate;

/* ------------------------------------------------------------ Definition 1 */
/* bit of qubit q in index x of an n-qubit register (qubit 0 = MSB) */
static inline int qbit(uint64_t x, int n, int q) {
    return (int)((x >> (unsigned)(n - 1 - q)) & 1u);
}
/* x with qubit q forced to v */
static inline uint64_t qforce(uint64_t x, int n, int q, int v) {
    uint64_t w = (uint64_t)1 << (unsigned)(n - 1 - q);
    return v ? (x | w) : (x & ~w);
}

static inline cplx mat(const double* m, int dim, int r, int c) {
    return m[2 * (r * dim + c)] + I * m[2 * (r * dim + c) + 1];
}

/* -------------------------------------------------- compensated summation */
typedef struct { double s, c; } nsum;
static inline void nsum_add(nsum* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nsum_get(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------ gate definitions */

/* psi = (I (x) U_q (x) I) phi, entry by entry */
void orc_apply_1q(int n, const double* in_, double* out_, int q, const double* u) {
    const cplx* in = (const cplx*)in_;
    cplx* out = (cplx*)out_;
    const uint64_t N = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t xi = 0; xi < (int64_t)N; ++xi) {
        uint64_t x = (uint64_t)xi;
        int r = qbit(x, n, q);
        cplx acc = 0;
        for (int c = 0; c < 2; ++c) acc += mat(u, 2, r, c) * in[qforce(x, n, q, c)];
        out[x] = acc;
    }
}

/* psi = |~cs><~cs|_qc (x) I + |cs><cs|_qc (x) U_qt, entry by entry */
void orc_apply_c1q(int n, const double* in_, double* out_, int qc, int qt, int cs,
                   const double* u) {
    const cplx* in = (const cplx*)in_;
    cplx* out = (cplx*)out_;
    const uint64_t N = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t xi = 0; xi < (int64_t)N; ++xi) {
        uint64_t x = (uint64_t)xi;
        if (qbit(x, n, qc) != cs) {
            out[x] = in[x];
            continue;
        }
        int r = qbit(x, n, qt);
        cplx acc = 0;
        for (int c = 0; c < 2; ++c) acc += mat(u, 2, r, c) * in[qforce(x, n, qt, c)];
        out[x] = acc;
    }
}

/* psi = U_{(qa,qb)} phi with local index 2*x_qa + x_qb, entry by entry */
void orc_apply_2q(int n, const double* in_, double* out_, int qa, int qb, const double* u) {
    const cplx* in = (const cplx*)in_;
    cplx* out = (cplx*)out_;
    const uint64_t N = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t xi = 0; xi < (int64_t)N; ++xi) {
        uint64_t x = (uint64_t)xi;
        int r = 2 * qbit(x, n, qa) + qbit(x, n, qb);
        cplx acc = 0;
        for (int c = 0; c < 4; ++c) {
            uint64_t y = qforce(qforce(x, n, qa, c >> 1), n, qb, c & 1);
            acc += mat(u, 4, r, c) * in[y];
        }
        out[x] = acc;
    }
}

/* psi = U_{(qs[0], .., qs[k-1])} phi for a 2^k x 2^k U (Sec. 2.4: a gate on
 * any k qubits, contiguous or not), entry by entry.  Row/column index
 * sum_i x_{qs[i]} 2^(k-1-i): qs[0] is the most significant local bit, which
 * is eq. (1)'s order when the qubits are contiguous and ascending. */
void orc_apply_kq(int n, const double* in_, double* out_, int k, const int* qs, const double* u) {
    const cplx* in = (const cplx*)in_;
    cplx* out = (cplx*)out_;
    const uint64_t N = (uint64_t)1 << n;
    const int dim = 1 << k;
#pragma omp parallel for schedule(static)
    for (int64_t xi = 0; xi < (int64_t)N; ++xi) {
        uint64_t x = (uint64_t)xi;
        int r = 0;
        for (int i = 0; i < k; ++i) r |= qbit(x, n, qs[i]) << (k - 1 - i);
        cplx acc = 0;
        for (int c = 0; c < dim; ++c) {
            uint64_t y = x;
            for (int i = 0; i < k; ++i) y = qforce(y, n, qs[i], (c >> (k - 1 - i)) & 1);
            acc += mat(u, dim, r, c) * in[y];
        }
        out[x] = acc;
    }
}

/* the Pauli matrices, row-major (re, im) pairs */
static const double PAULI[3][8] = {
    {0, 0, 1, 0, 1, 0, 0, 0},     /* X = [[0,1],[1,0]] */
    {0, 0, 0, -1, 0, 1, 0, 0},    /* Y = [[0,-i],[i,0]] */
    {1, 0, 0, 0, 0, 0, -1, 0},    /* Z = [[1,0],[0,-1]] */
};

/* exp(-i theta P / 2) = cos(theta/2) I - i sin(theta/2) P */
void orc_rotation(int axis, double theta, double* u) {
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    for (int k = 0; k < 4; ++k) {
        cplx p = PAULI[axis][2 * k] + I * PAULI[axis][2 * k + 1];
        cplx e = (k == 0 || k == 3 ? c : 0.0) - I * s * p;
        u[2 * k] = creal(e);
        u[2 * k + 1] = cimag(e);
    }
}

static void pauli_matrix(int axis, double* u) { memcpy(u, PAULI[axis], 8 * sizeof(double)); }

static void adjoint2(const double* u, double* ud) {
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            ud[2 * (r * 2 + c)] = u[2 * (c * 2 + r)];
            ud[2 * (r * 2 + c) + 1] = -u[2 * (c * 2 + r) + 1];
        }
}
static void adjoint4(const double* u, double* ud) {
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            ud[2 * (r * 4 + c)] = u[2 * (c * 4 + r)];
            ud[2 * (r * 4 + c) + 1] = -u[2 * (c * 4 + r) + 1];
        }
}

/* Extra controls (Sec. 2.4, Fig. 5: a multi-controlled gate acts only where
 * every control qubit holds its value):
 *     P_c (x) U + (I - P_c) (x) I,   P_c = prod_{q in cmask} |v_q><v_q|_q.
 * Entry by entry: out[x] is the gate's result where x satisfies the
 * controls, and in[x] elsewhere.  The gate's own entries only combine
 * amplitudes that differ in its own qubits, so a satisfied x only reads
 * amplitudes that satisfy the controls too. */
static int controls_hold(int n, uint64_t x, uint64_t cmask, uint64_t cvals) {
    for (int q = 0; q < n; ++q)
        if (((cmask >> q) & 1u) && qbit(x, n, q) != (int)((cvals >> q) & 1u)) return 0;
    return 1;
}
static void keep_unselected(int n, const double* in_, double* out_, uint64_t cmask, uint64_t cvals) {
    const cplx* in = (const cplx*)in_;
    cplx* out = (cplx*)out_;
    const uint64_t N = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t xi = 0; xi < (int64_t)N; ++xi)
        if (!controls_hold(n, (uint64_t)xi, cmask, cvals)) out[xi] = in[xi];
}

/* Apply gate g (or its adjoint) from in to out. */
static void apply_gate(int n, const double* in, double* out, const orc_gate* g,
                       const double* params, int dagger) {
    double u[32], ud[32];
    switch (g->kind) {
    case ORC_1Q:
        if (dagger) { adjoint2(g->m, ud); orc_apply_1q(n, in, out, g->q0, ud); }
        else orc_apply_1q(n, in, out, g->q0, g->m);
        break;
    case ORC_C1Q:
        if (dagger) { adjoint2(g->m, ud); orc_apply_c1q(n, in, out, g->q0, g->q1, g->ctrl_state, ud); }
        else orc_apply_c1q(n, in, out, g->q0, g->q1, g->ctrl_state, g->m);
        break;
    case ORC_2Q:
        if (dagger) { adjoint4(g->m, ud); orc_apply_2q(n, in, out, g->q0, g->q1, ud); }
        else orc_apply_2q(n, in, out, g->q0, g->q1, g->m);
        break;
    case ORC_ROT:
        orc_rotation(g->axis, dagger ? -params[g->param] : params[g->param], u);
        orc_apply_1q(n, in, out, g->q0, u);
        break;
    }
    if (g->cmask) keep_unselected(n, in, out, g->cmask, g->cvals);
}

/* Run gates [0, ng) on state (in place from the caller's view); work is a
 * second buffer of the same size. */
void orc_run(int n, double* state, double* work, int64_t ng, const orc_gate* gates,
             const double* params) {
    const size_t bytes = ((size_t)1 << n) * 2 * sizeof(double);
    double* a = state;
    double* b = work;
    for (int64_t k = 0; k < ng; ++k) {
        apply_gate(n, a, b, &gates[k], params, 0);
        double* t = a; a = b; b = t;
    }
    if (a != state) memcpy(state, a, bytes);
}

/* state = |basis> */
void orc_init_basis(int n, double* state, uint64_t basis) {
    const size_t N = (size_t)1 << n;
    memset(state, 0, N * 2 * sizeof(double));
    state[2 * basis] = 1.0;
}

/* ------------------------------------------------------------ reductions */

double orc_norm2(int n, const double* s_) {
    const cplx* s = (const cplx*)s_;
    nsum acc = {0, 0};
    for (uint64_t x = 0; x < ((uint64_t)1 << n); ++x) {
        nsum_add(&acc, creal(s[x]) * creal(s[x]));
        nsum_add(&acc, cimag(s[x]) * cimag(s[x]));
    }
    return nsum_get(&acc);
}

/* <Z^{qmask}> = sum_x |s_x|^2 prod_{q in qmask} (-1)^{x_q};  qmask bit q = qubit q */
double orc_expect_z(int n, const double* s_, uint64_t qmask) {
    const cplx* s = (const cplx*)s_;
    nsum acc = {0, 0};
    for (uint64_t x = 0; x < ((uint64_t)1 << n); ++x) {
        int sign = 1;
        for (int q = 0; q < n; ++q)
            if (((qmask >> q) & 1u) && qbit(x, n, q)) sign = -sign;
        double p = creal(s[x]) * creal(s[x]) + cimag(s[x]) * cimag(s[x]);
        nsum_add(&acc, sign * p);
    }
    return nsum_get(&acc);
}

/* <a|b> = sum_x conj(a_x) b_x */
void orc_inner(int n, const double* a_, const double* b_, double* out) {
    const cplx* a = (const cplx*)a_;
    const cplx* b = (const cplx*)b_;
    nsum re = {0, 0}, im = {0, 0};
    for (uint64_t x = 0; x < ((uint64_t)1 << n); ++x) {
        cplx t = conj(a[x]) * b[x];
        nsum_add(&re, creal(t));
        nsum_add(&im, cimag(t));
    }
    out[0] = nsum_get(&re);
    out[1] = nsum_get(&im);
}

/* P(qubit q measures 1) = sum over x with x_q = 1 of |s_x|^2 */
double orc_prob1(int n, const double* s_, int q) {
    const cplx* s = (const cplx*)s_;
    nsum acc = {0, 0};
    for (uint64_t x = 0; x < ((uint64_t)1 << n); ++x)
        if (qbit(x, n, q))
            nsum_add(&acc, creal(s[x]) * creal(s[x]) + cimag(s[x]) * cimag(s[x]));
    return nsum_get(&acc);
}

/* Projective measurement of qubit q with uniform draw r in [0,1): outcome 0
 * iff r < P(0); the state is projected onto the outcome and renormalised. */
int orc_measure1(int n, double* s_, int q, double r) {
    cplx* s = (cplx*)s_;
    double p1 = orc_prob1(n, s_, q);
    double p0 = orc_norm2(n, s_) - p1;
    int outcome = (r < p0) ? 0 : 1;
    double keep = outcome ? p1 : p0;
    double scale = 1.0 / sqrt(keep);
    for (uint64_t x = 0; x < ((uint64_t)1 << n); ++x)
        s[x] = (qbit(x, n, q) == outcome) ? s[x] * scale : 0.0;
    return outcome;
}

/* ----------------------------------------------------------- observables */

/* O = sum_k w_k Z^{qmask_k}; returns <s|O|s> */
double orc_expect_obs(int n, const double* s, int nterms, const uint64_t* qmasks,
                      const double* w) {
    double e = 0.0;
    for (int k = 0; k < nterms; ++k) e += w[k] * orc_expect_z(n, s, qmasks[k]);
    return e;
}

/* out = O s for diagonal O = sum_k w_k Z^{qmask_k} */
static void apply_obs(int n, const double* s_, double* out_, int nterms, const uint64_t* qmasks,
                      const double* w) {
    const cplx* s = (const cplx*)s_;
    cplx* out = (cplx*)out_;
#pragma omp parallel for schedule(static)
    for (int64_t xi = 0; xi < ((int64_t)1 << n); ++xi) {
        uint64_t x = (uint64_t)xi;
        double d = 0.0;
        for (int k = 0; k < nterms; ++k) {
            int sign = 1;
            for (int q = 0; q < n; ++q)
                if (((qmasks[k] >> q) & 1u) && qbit(x, n, q)) sign = -sign;
            d += w[k] * sign;
        }
        out[x] = d * s[x];
    }
}

/* f(params) = <0| U^dagger O U |0> for the circuit; scratch: two state buffers */
double orc_energy(int n, int64_t ng, const orc_gate* gates, const double* params, int nterms,
                  const uint64_t* qmasks, const double* w, double* s, double* work) {
    orc_init_basis(n, s, 0);
    orc_run(n, s, work, ng, gates, params);
    return orc_expect_obs(n, s, nterms, qmasks, w);
}

/*
 * Adjoint-method gradient (Jones & Gacon): with psi = U_P..U_1|0>,
 * lambda = O psi, walk k = P..1: if gate k is exp(-i theta P_k / 2) with
 * parameter j, grad[j] += Im <lambda| P_k |psi>; then psi <- U_k^dag psi and
 * lambda <- U_k^dag lambda.  Buffers: psi, lam, tmp each 2^n complex.
 */
double orc_adjoint(int n, int64_t ng, const orc_gate* gates, const double* params, int nparams,
                   int nterms, const uint64_t* qmasks, const double* w, double* grad,
                   double* psi, double* lam, double* tmp) {
    const size_t bytes = ((size_t)1 << n) * 2 * sizeof(double);
    for (int j = 0; j < nparams; ++j) grad[j] = 0.0;
    orc_init_basis(n, psi, 0);
    orc_run(n, psi, tmp, ng, gates, params);
    double f = orc_expect_obs(n, psi, nterms, qmasks, w);
    apply_obs(n, psi, lam, nterms, qmasks, w);
    for (int64_t k = ng - 1; k >= 0; --k) {
        const orc_gate* g = &gates[k];
        if (g->kind == ORC_ROT) {
            double p[8], ip[2];
            pauli_matrix(g->axis, p);
            orc_apply_1q(n, psi, tmp, g->q0, p);     /* tmp = P psi */
            orc_inner(n, lam, tmp, ip);              /* <lam| P psi> */
            grad[g->param] += ip[1];
        }
        apply_gate(n, psi, tmp, g, params, 1);
        memcpy(psi, tmp, bytes);
        apply_gate(n, lam, tmp, g, params, 1);
        memcpy(lam, tmp, bytes);
    }
    return f;
}

/* Parameter shift: grad[j] = (f(theta_j + pi/2) - f(theta_j - pi/2)) / 2, for
 * each listed parameter j (each parameter must drive a single rotation). */
void orc_param_shift(int n, int64_t ng, const orc_gate* gates, const double* params, int nparams,
                     int nsel, const int* sel, int nterms, const uint64_t* qmasks,
                     const double* w, double* grad_sel, double* s, double* work) {
    double* p = (double*)malloc(sizeof(double) * (size_t)(nparams > 0 ? nparams : 1));
    memcpy(p, params, sizeof(double) * (size_t)nparams);
    for (int i = 0; i < nsel; ++i) {
        int j = sel[i];
        p[j] = params[j] + 0.5 * ORC_PI;
        double fp = orc_energy(n, ng, gates, p, nterms, qmasks, w, s, work);
        p[j] = params[j] - 0.5 * ORC_PI;
        double fm = orc_energy(n, ng, gates, p, nterms, qmasks, w, s, work);
        p[j] = params[j];
        grad_sel[i] = 0.5 * (fp - fm);
    }
    free(p);
}

/* Central finite differences with step h for the listed parameters. */
void orc_finite_diff(int n, int64_t ng, const orc_gate* gates, const double* params, int nparams,
                     int nsel, const int* sel, double h, int nterms, const uint64_t* qmasks,
                     const double* w, double* grad_sel, double* s, double* work) {
    double* p = (double*)malloc(sizeof(double) * (size_t)(nparams > 0 ? nparams : 1));
    memcpy(p, params, sizeof(double) * (size_t)nparams);
    for (int i = 0; i < nsel; ++i) {
        int j = sel[i];
        p[j] = params[j] + h;
        double fp = orc_energy(n, ng, gates, p, nterms, qmasks, w, s, work);
        p[j] = params[j] - h;
        double fm = orc_energy(n, ng, gates, p, nterms, qmasks, w, s, work);
        p[j] = params[j];
        grad_sel[i] = (fp - fm) / (2.0 * h);
    }
    free(p);
}

/* Amplitude <x| (tensor product of single-qubit states) : for product-state
 * checks.  qstates[2*q..] is qubit q's 2-vector (re,im pairs: 4 doubles). */
void orc_product_amplitude(int n, const double* qstates, uint64_t x, double* out) {
    cplx a = 1.0;
    for (int q = 0; q < n; ++q) {
        int v = qbit(x, n, q);
        a *= qstates[4 * q + 2 * v] + I * qstates[4 * q + 2 * v + 1];
    }
    out[0] = creal(a);
    out[1] = cimag(a);
}

/* Thread count of the OpenMP loops (the benchmark's CPU baseline times the
 * oracle on one thread and on every core). */
void orc_set_num_threads(int t) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
