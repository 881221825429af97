"""Pins for the FP64 CPU oracle, independent of the oracle's own formulas.

Each check ties the oracle to something the paper or the mathematics fixes:
the worked index examples of Figs. 3-5, dense Kronecker products built with
numpy.kron (eq. (1) taken literally), tensor contractions with numpy, the
closed forms of Sec. 2 (Pauli X/Y/Z, CNOT, SWAP), the QFT of Fig. 1 against
numpy's FFT, and analytic expectation values and gradients.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W
from oracle import indices as IX

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _rand_state(n, seed):
    return W.random_state(n, seed)


# ------------------------------------------------ dense Kronecker operators
def kron_all(*ms):
    out = np.eye(1, dtype=np.complex128)
    for m in ms:
        out = np.kron(out, m)
    return out


def dense_1q(n, q, u):
    """I_{2^q} (x) U (x) I_{2^(n-q-1)}: eq. (1) with qubit 0 leftmost."""
    return kron_all(np.eye(2 ** q), u, np.eye(2 ** (n - q - 1)))


def dense_adjacent_2q(n, q, u):
    """U on the contiguous pair (q, q+1), basis 2*x_q + x_{q+1}."""
    return kron_all(np.eye(2 ** q), u, np.eye(2 ** (n - q - 2)))


def dense_2q(n, qa, qb, u):
    """U on (qa, qb), local index 2*x_qa + x_qb, built only from kron products:
    move qb next to qa by adjacent SWAPs, apply the contiguous operator, move
    back.  For qa > qb the matrix is first conjugated by SWAP so the lower
    qubit comes first."""
    if qa > qb:
        u = W.SWAP @ u @ W.SWAP
        qa, qb = qb, qa
    chain = np.eye(2 ** n, dtype=np.complex128)
    for p in range(qb - 1, qa, -1):       # swap (p, p+1) moves qb down to qa+1
        chain = dense_adjacent_2q(n, p, W.SWAP) @ chain
    return chain.conj().T @ dense_adjacent_2q(n, qa, u) @ chain


def dense_c1q(n, qc, qt, u, cs):
    """|~cs><~cs|_qc (x) I + |cs><cs|_qc (x) U_qt via kron products."""
    proj = [np.diag([1.0, 0.0]).astype(np.complex128), np.diag([0.0, 1.0]).astype(np.complex128)]
    factors_on = [np.eye(2, dtype=np.complex128)] * n
    factors_off = [np.eye(2, dtype=np.complex128)] * n
    factors_on = list(factors_on)
    factors_off = list(factors_off)
    factors_on[qc] = proj[cs]
    factors_on[qt] = u
    factors_off[qc] = proj[1 - cs]
    return kron_all(*factors_on) + kron_all(*factors_off)


# ------------------------------------------------ tensor-contraction helper
def tensor_apply(state, qubits, u):
    """Apply a k-qubit gate by contracting the (2,)*n tensor; C order puts
    qubit 0 on axis 0, which is Definition 1."""
    n = int(np.log2(state.size))
    k = len(qubits)
    t = state.reshape((2,) * n)
    ut = u.reshape((2,) * (2 * k))
    t = np.tensordot(ut, t, axes=(list(range(k, 2 * k)), list(qubits)))
    # result axes: gate outputs first, then the remaining axes in order
    rest = [a for a in range(n) if a not in qubits]
    order = list(qubits) + rest
    inv = np.argsort(order)
    return np.transpose(t, inv).reshape(-1)


# ============================================================ index pins
def test_fig3_index_sets():
    g = _gold("fig3_1q_n3.json")
    for case in g["cases"]:
        m_l, m_r = IX.masks_1q(g["n"], case["q"])
        assert (m_l, m_r) == (case["mL"], case["mR"])
        pairs = IX.pairs_1q(g["n"], case["q"])
        assert [a for a, _ in pairs] == case["a"]
        assert [b for _, b in pairs] == case["b"]


def test_fig4_index_sets():
    g = _gold("fig4_c1q_n3.json")
    for case in g["cases"]:
        pairs = IX.pairs_c1q(g["n"], case["qc"], case["qt"], case["cs"])
        assert [a for a, _ in pairs] == case["a"]
        assert [b for _, b in pairs] == case["b"]


def test_fig5_doubly_controlled_set():
    """Two controls: pairs of the C1q map on (q1 -> q2) restricted to q0 = 1."""
    g = _gold("fig5_cc1q_n3.json")
    n = g["n"]
    c0, c1 = g["controls"]
    pairs = IX.pairs_c1q(n, c1, g["target"], 1)
    w0 = 2 ** (n - c0 - 1)
    sel = [(a, b) for a, b in pairs if a & w0]
    assert [a for a, _ in sel] == g["a"]
    assert [b for _, b in sel] == g["b"]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10])
def test_partition_1q(n):
    full = set(range(2 ** n))
    for q in range(n):
        seen = [i for p in IX.pairs_1q(n, q) for i in p]
        assert len(seen) == 2 ** n and set(seen) == full
        for a, b in IX.pairs_1q(n, q):
            assert b - a == 2 ** (n - q - 1) and not (a >> (n - q - 1)) & 1


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_partition_c1q_and_2q(n):
    full = set(range(2 ** n))
    for qa in range(n):
        for qb in range(n):
            if qa == qb:
                continue
            both = [i for cs in (0, 1) for p in IX.pairs_c1q(n, qa, qb, cs) for i in p]
            half = set(i for p in IX.pairs_c1q(n, qa, qb, 1) for i in p)
            # control-1 pairs cover exactly the indices with the control bit set
            assert half == {x for x in full if (x >> (n - qa - 1)) & 1}
            assert len(both) == 2 ** n and set(both) == full
            quads = [i for p in IX.quads_2q(n, qa, qb) for i in p]
            assert len(quads) == 2 ** n and set(quads) == full


# ====================================================== gate values vs kron
@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_oracle_1q_vs_kron(n):
    rng = np.random.default_rng(10 + n)
    phi = _rand_state(n, 100 + n)
    for q in range(n):
        u = W.haar_unitary(2, rng)
        ref = dense_1q(n, q, u) @ phi
        got = O.apply_1q(phi, q, u)
        assert np.max(np.abs(got - ref)) < 1e-14
        assert np.max(np.abs(tensor_apply(phi, [q], u) - ref)) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_oracle_c1q_vs_kron(n):
    rng = np.random.default_rng(20 + n)
    phi = _rand_state(n, 200 + n)
    for qc in range(n):
        for qt in range(n):
            if qc == qt:
                continue
            for cs in (0, 1):
                u = W.haar_unitary(2, rng)
                ref = dense_c1q(n, qc, qt, u, cs) @ phi
                got = O.apply_c1q(phi, qc, qt, u, cs)
                assert np.max(np.abs(got - ref)) < 1e-14, (qc, qt, cs)


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_oracle_2q_vs_kron(n):
    rng = np.random.default_rng(30 + n)
    phi = _rand_state(n, 300 + n)
    for qa in range(n):
        for qb in range(n):
            if qa == qb:
                continue
            u = W.haar_unitary(4, rng)
            ref = dense_2q(n, qa, qb, u) @ phi
            got = O.apply_2q(phi, qa, qb, u)
            assert np.max(np.abs(got - ref)) < 1e-14, (qa, qb)
            assert np.max(np.abs(tensor_apply(phi, [qa, qb], u) - ref)) < 1e-14


def test_2q_local_order_contiguous_is_kron():
    """For a contiguous pair, eq. (1) fixes the local order: a 2q gate equal
    to A (x) B on (q, q+1) acts as A on q and B on q+1."""
    rng = np.random.default_rng(5)
    n = 5
    phi = _rand_state(n, 55)
    a, b = W.haar_unitary(2, rng), W.haar_unitary(2, rng)
    for q in range(n - 1):
        got = O.apply_2q(phi, q, q + 1, np.kron(a, b))
        ref = O.apply_1q(O.apply_1q(phi, q, a), q + 1, b)
        assert np.max(np.abs(got - ref)) < 1e-14


def test_2q_product_gate_any_pair():
    rng = np.random.default_rng(6)
    n = 6
    phi = _rand_state(n, 66)
    for qa in range(n):
        for qb in range(n):
            if qa == qb:
                continue
            a, b = W.haar_unitary(2, rng), W.haar_unitary(2, rng)
            got = O.apply_2q(phi, qa, qb, np.kron(a, b))
            ref = tensor_apply(tensor_apply(phi, [qa], a), [qb], b)
            assert np.max(np.abs(got - ref)) < 1e-14


def test_alg3_as_printed_disagrees_with_eq1():
    """Alg. 3 as printed pairs row 1 of U with q0's bit set; eq. (1) puts
    q1's bit there for a contiguous pair.  The two agree only for gates
    symmetric under exchanging the qubits (e.g. SWAP, the printed example)."""
    rng = np.random.default_rng(7)
    n, q0, q1 = 3, 0, 1
    phi = _rand_state(n, 77)
    u = W.haar_unitary(4, rng)
    literal = phi.copy()
    for quad in IX.quads_2q_as_printed(n, q0, q1):
        v = phi[list(quad)]
        literal[list(quad)] = u @ v
    ref = dense_adjacent_2q(n, q0, u) @ phi
    assert np.max(np.abs(literal - ref)) > 1e-3
    ours = phi.copy()
    for quad in IX.quads_2q(n, q0, q1):
        ours[list(quad)] = u @ phi[list(quad)]
    assert np.max(np.abs(ours - ref)) < 1e-14
    sw = phi.copy()
    for quad in IX.quads_2q_as_printed(n, q0, q1):
        sw[list(quad)] = W.SWAP @ phi[list(quad)]
    assert np.max(np.abs(sw - dense_adjacent_2q(n, q0, W.SWAP) @ phi)) < 1e-15


# ============================================= closed forms of Sec. 2
@pytest.mark.parametrize("n", [1, 3, 6])
def test_pauli_closed_forms(n):
    """Sec. 2.1: X swaps a_j and b_j; Y maps (a,b) -> (-i b, i a); Z negates b."""
    phi = _rand_state(n, 400 + n)
    for q in range(n):
        pairs = IX.pairs_1q(n, q)
        a = np.array([p[0] for p in pairs])
        b = np.array([p[1] for p in pairs])
        x = O.apply_1q(phi, q, W.X)
        assert np.array_equal(x[a], phi[b]) and np.array_equal(x[b], phi[a])
        y = O.apply_1q(phi, q, W.Y)
        assert np.allclose(y[a], -1j * phi[b], atol=0, rtol=0) and np.allclose(y[b], 1j * phi[a], atol=0, rtol=0)
        z = O.apply_1q(phi, q, W.Z)
        assert np.array_equal(z[a], phi[a]) and np.array_equal(z[b], -phi[b])


def test_hzh_is_x():
    phi = _rand_state(4, 9)
    for q in range(4):
        s = O.apply_1q(O.apply_1q(O.apply_1q(phi, q, W.H), q, W.Z), q, W.H)
        assert np.max(np.abs(s - O.apply_1q(phi, q, W.X))) < 1e-15


def test_cnot_squared_is_identity_and_swaps_half():
    """Sec. 2.2: CNOT only swaps half the elements; CNOT.CNOT = I."""
    n = 5
    phi = _rand_state(n, 11)
    for qc in range(n):
        for qt in range(n):
            if qc == qt:
                continue
            s = O.apply_c1q(phi, qc, qt, W.X, 1)
            changed = np.nonzero(s != phi)[0]
            assert len(changed) == 2 ** (n - 1)
            for a, b in IX.pairs_c1q(n, qc, qt, 1):
                assert s[a] == phi[b] and s[b] == phi[a]
            assert np.array_equal(O.apply_c1q(s, qc, qt, W.X, 1), phi)


def test_swap_closed_form():
    """Sec. 2.3: SWAP keeps a_j, d_j and exchanges b_j, c_j."""
    n = 5
    phi = _rand_state(n, 12)
    for q0 in range(n):
        for q1 in range(q0 + 1, n):
            s = O.apply_2q(phi, q0, q1, W.SWAP)
            for a, b, c, d in IX.quads_2q_as_printed(n, q0, q1):
                assert s[a] == phi[a] and s[d] == phi[d]
                assert s[b] == phi[c] and s[c] == phi[b]


def test_bell_and_ghz():
    s = O.basis(2)
    s = O.apply_1q(s, 0, W.H)
    s = O.apply_c1q(s, 0, 1, W.X, 1)
    assert np.allclose(s, np.array([1, 0, 0, 1]) / np.sqrt(2), atol=1e-16)
    for n in (3, 6, 9):
        s = O.basis(n)
        s = O.apply_1q(s, 0, W.H)
        for q in range(n - 1):
            s = O.apply_c1q(s, q, q + 1, W.X, 1)
        ref = np.zeros(2 ** n, dtype=complex)
        ref[0] = ref[-1] = 1 / np.sqrt(2)
        assert np.max(np.abs(s - ref)) < 1e-15
        for i in range(n):
            assert abs(O.expect_z(s, [i])) < 1e-15
            for j in range(i + 1, n):
                assert abs(O.expect_z(s, [i, j]) - 1.0) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_qft_is_fft(n):
    """The QFT circuit of Fig. 1 (theta = -2 pi / 2^j as printed) maps any
    state to numpy.fft.fft(phi)/sqrt(N)."""
    phi = _rand_state(n, 500 + n)
    got = O.run(W.qft(n), phi)
    ref = np.fft.fft(phi) / np.sqrt(2 ** n)
    assert np.max(np.abs(got - ref)) < 1e-13
    zero = O.run(W.qft(n))
    assert np.max(np.abs(zero - 1 / np.sqrt(2 ** n))) < 1e-14


# ====================================================== rotations & runs
@pytest.mark.parametrize("axis,p", [("X", W.X), ("Y", W.Y), ("Z", W.Z)])
def test_rotation_is_matrix_exponential(axis, p):
    for theta in (0.0, 0.3, -1.7, 2.5, 6.0):
        ref = scipy.linalg.expm(-0.5j * theta * p)
        assert np.max(np.abs(O.rotation(axis, theta) - ref)) < 1e-15


def test_run_matches_kron_product():
    """A whole circuit equals the product of its dense operators."""
    n = 5
    c = W.random_mix(n, 40, seed=3)
    m = np.eye(2 ** n, dtype=np.complex128)
    for g in c.gates:
        if g.kind == W.KIND_1Q:
            d = dense_1q(n, g.qubits[0], g.matrix)
        elif g.kind == W.KIND_C1Q:
            d = dense_c1q(n, g.qubits[0], g.qubits[1], g.matrix, g.ctrl_state)
        else:
            d = dense_2q(n, g.qubits[0], g.qubits[1], g.matrix)
        m = d @ m
    phi = _rand_state(n, 13)
    assert np.max(np.abs(O.run(c, phi) - m @ phi)) < 1e-13


def test_inverse_circuit_returns_state():
    c = W.mix_n10_g200()
    phi = _rand_state(c.n, 14)
    s = O.run(W.inverse(c), O.run(c, phi))
    assert np.max(np.abs(s - phi)) < 1e-12


# ============================================================ reductions
def test_z_on_basis_states():
    """<Z_q> on |b> is +1 when bit q of b (Definition 1) is 0, else -1."""
    n = 6
    for b in (0, 1, 5, 37, 63):
        s = O.basis(n, b)
        for q in range(n):
            bit = (b >> (n - 1 - q)) & 1
            assert O.expect_z(s, [q]) == (1.0 if bit == 0 else -1.0)
            assert O.prob1(s, q) == float(bit)


def test_ry_expectation_cos():
    for theta in (0.0, 0.4, 1.0, 2.9, 4.4):
        s = O.apply_1q(O.basis(1), 0, O.rotation("Y", theta))
        assert abs(O.expect_z(s, [0]) - np.cos(theta)) < 1e-15


def test_norm_inner_prob_vs_numpy():
    n = 9
    a, b = _rand_state(n, 15), _rand_state(n, 16)
    assert abs(O.norm2(a) - 1.0) < 1e-14
    v = O.inner(a, b)
    assert abs(v - np.vdot(a, b)) < 1e-14
    t = a.reshape((2,) * n)
    for q in range(n):
        p1 = np.sum(np.abs(np.take(t, 1, axis=q)) ** 2)
        assert abs(O.prob1(a, q) - p1) < 1e-14
    for qs in ([0], [3, 8], [0, 4, 5]):
        signs = np.ones(2 ** n)
        for q in qs:
            bits = (np.arange(2 ** n) >> (n - 1 - q)) & 1
            signs *= 1 - 2 * bits
        assert abs(O.expect_z(a, qs) - np.sum(signs * np.abs(a) ** 2)) < 1e-14


def test_norm_preserved_by_circuit():
    c = W.mix_n10_g200()
    assert abs(O.norm2(O.run(c)) - 1.0) < 1e-13


def test_measure_collapse():
    n = 5
    s = _rand_state(n, 17)
    for q in range(n):
        p1 = O.prob1(s, q)
        for r, expect in ((0.5 * (1 - p1), 0), (1 - 0.5 * p1, 1)):
            k, post = O.measure1(s, q, r)
            assert k == expect
            t = post.reshape((2,) * n)
            assert np.all(np.take(t, 1 - k, axis=q) == 0)
            assert abs(O.norm2(post) - 1.0) < 1e-14
            keep = np.take(s.reshape((2,) * n), k, axis=q)
            assert np.allclose(np.take(t, k, axis=q), keep / np.linalg.norm(keep), atol=1e-15)


def test_product_amplitude_vs_kron():
    rng = np.random.default_rng(18)
    qs = np.array([W.haar_unitary(2, rng)[:, 0] for _ in range(6)])
    full = kron_all(*[q.reshape(2, 1) for q in qs]).reshape(-1)
    for x in (0, 1, 17, 63):
        assert abs(O.product_amplitude(qs, x) - full[x]) < 1e-15


# ============================================================ gradients
def test_single_ry_gradient_closed_form():
    """f = <0|RY(t)^dag Z RY(t)|0> = cos t, df/dt = -sin t."""
    for t in (0.1, 1.3, 2.2, 5.0):
        c = W.Circuit(1, [W.grot(0, "Y", 0)], np.array([t]), [((0,), 1.0)])
        f, g = O.adjoint(c)
        assert abs(f - np.cos(t)) < 1e-15
        assert abs(g[0] + np.sin(t)) < 1e-15
        assert abs(O.param_shift(c)[0] + np.sin(t)) < 1e-15


def test_rx_rz_gradient_closed_form():
    """RX(a) then RZ(b) on |0>: <Z> = cos a (independent of b); <X> after RY
    would depend on both -- check the Z part and a two-qubit product."""
    a, b = 0.7, 1.9
    c = W.Circuit(2, [W.grot(0, "X", 0), W.grot(1, "Y", 1)], np.array([a, b]),
                  [((0, 1), 1.0)])
    f, g = O.adjoint(c)
    assert abs(f - np.cos(a) * np.cos(b)) < 1e-15
    assert abs(g[0] + np.sin(a) * np.cos(b)) < 1e-15
    assert abs(g[1] + np.cos(a) * np.sin(b)) < 1e-15


@pytest.mark.parametrize("n,layers", [(3, 2), (5, 3)])
def test_adjoint_vs_shift_vs_fd(n, layers):
    c = W.hea_cz_ring(n, layers, seed=19 + n)
    f, g = O.adjoint(c)
    assert abs(f - O.energy(c)) < 1e-13
    ps = O.param_shift(c)
    fd = O.finite_diff(c, h=1e-6)
    wsum = sum(abs(w) for _, w in c.observable)
    assert np.max(np.abs(g - ps)) < 1e-12 * max(1, wsum)
    assert np.max(np.abs(g - fd)) < 1e-6 * max(1, wsum)


def test_ry_rz_ladder_gradients():
    rng = np.random.default_rng(21)
    c = W.ry_rz_cnot_ladder(4, 2, rng)
    f, g = O.adjoint(c)
    assert np.max(np.abs(g - O.param_shift(c))) < 1e-12


# ------------------------------------ gradients through general fixed gates
_PAULI = {"X": W.X, "Y": W.Y, "Z": W.Z}


def _dense_gate(n, g, params):
    """Dense operator of one gate from kron products alone (eq. (1) literally;
    rotations as matrix exponentials of their Pauli generator)."""
    if g.kind == W.KIND_ROT:
        u = scipy.linalg.expm(-0.5j * params[g.param] * _PAULI[g.axis])
        return dense_1q(n, g.qubits[0], u)
    if g.kind == W.KIND_1Q:
        return dense_1q(n, g.qubits[0], g.matrix)
    if g.kind == W.KIND_C1Q:
        return dense_c1q(n, g.qubits[0], g.qubits[1], g.matrix, g.ctrl_state)
    return dense_2q(n, g.qubits[0], g.qubits[1], g.matrix)


def _dense_energy_and_grad(c):
    """f = <0|U^dag O U|0> and df/dtheta_j from dense products:
    d/dtheta exp(-i theta P/2) = (-i/2) P exp(-i theta P/2), carried through
    the rest of the circuit as a second vector; df = 2 Re <psi| O |dpsi>."""
    n = c.n
    mats = [_dense_gate(n, g, c.params) for g in c.gates]
    diag = np.zeros(2 ** n)
    for qs, w in c.observable:
        ops = [W.Z if q in qs else W.I2 for q in range(n)]
        diag += w * np.real(np.diag(kron_all(*ops)))
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    prefix = []
    for m in mats:
        prefix.append(psi)
        psi = m @ psi
    grad = np.zeros(c.params.size)
    for k, g in enumerate(c.gates):
        if g.kind != W.KIND_ROT:
            continue
        d = dense_1q(n, g.qubits[0], -0.5j * _PAULI[g.axis]) @ (mats[k] @ prefix[k])
        for m in mats[k + 1:]:
            d = m @ d
        grad[g.param] += 2.0 * np.real(np.vdot(psi, diag * d))
    return float(np.real(np.vdot(psi, diag * psi))), grad


@pytest.mark.parametrize("n,layers,seed", [(4, 2, 31), (5, 2, 32), (6, 1, 33)])
def test_adjoint_through_general_fixed_gates(n, layers, seed):
    """The adjoint sweep rewinds every fixed gate with its conjugate
    transpose.  With Haar 1q, Haar 2q (both qubit orders) and controlled Haar
    gates (control state 0 and 1) in the circuit, a missing conjugation or
    transposition in that rewind changes the gradient; the dense-matrix
    derivative above and the parameter-shift rule (forward runs only) both
    pin it."""
    c = W.mixed_param_circuit(n, layers, seed)
    kinds = {(g.kind, g.ctrl_state if g.kind == W.KIND_C1Q else None) for g in c.gates}
    assert {(W.KIND_1Q, None), (W.KIND_2Q, None), (W.KIND_C1Q, 0), (W.KIND_C1Q, 1)} <= kinds
    assert any(g.kind == W.KIND_2Q and g.qubits[0] > g.qubits[1] for g in c.gates)
    for g in c.gates:   # none of the fixed gates is its own adjoint
        if g.kind != W.KIND_ROT:
            assert np.max(np.abs(g.matrix - g.matrix.conj().T)) > 1e-3
    f_ref, g_ref = _dense_energy_and_grad(c)
    f, g = O.adjoint(c)
    wsum = max(1.0, sum(abs(w) for _, w in c.observable))
    assert abs(f - f_ref) < 1e-13 * wsum
    assert np.max(np.abs(g - g_ref)) < 1e-12 * wsum
    assert np.max(np.abs(O.param_shift(c) - g_ref)) < 1e-12 * wsum
    assert np.max(np.abs(O.finite_diff(c, h=1e-6) - g_ref)) < 1e-6 * wsum


# ------------------------------------------- Trotter (Hamiltonian) circuit
def test_trotter_block_is_xx_zz_exponential():
    """CNOT . (RX(a) on the control, RZ(b) on the target) . CNOT equals
    exp(-i a/2 X(x)X) exp(-i b/2 Z(x)Z): conjugation by CNOT maps X(x)I to
    X(x)X and I(x)Z to Z(x)Z.  The oracle runs the gate sequence; the closed
    form is two matrix exponentials."""
    a, b = 0.83, 2.41
    XX = np.kron(W.X, W.X)
    ZZ = np.kron(W.Z, W.Z)
    ref_op = scipy.linalg.expm(-0.5j * a * XX) @ scipy.linalg.expm(-0.5j * b * ZZ)
    c = W.Circuit(2, [W.cnot(0, 1), W.grot(0, "X", 0), W.grot(1, "Z", 1), W.cnot(0, 1)],
                  np.array([a, b]))
    for seed in (1, 2, 3):
        s = _rand_state(2, 300 + seed)
        assert np.max(np.abs(O.run(c, state=s) - ref_op @ s)) < 1e-15


@pytest.mark.parametrize("n,steps", [(4, 2), (5, 1), (6, 2)])
def test_trotter_circuit_vs_dense(n, steps):
    """The Trotter generator's circuit through the oracle against the product
    of its gates' dense kron operators; its layout follows the figure: two
    RZ columns and four gates per nearest-neighbour pair per step, then a
    closing RZ on the odd-block qubits."""
    c = W.trotter_tfxy(n, steps, seed=40 + n)
    npairs = n - 1
    assert len(c.gates) == steps * (2 * n + 4 * npairs) + 2 * ((n - 1) // 2)
    assert c.params.size == sum(g.kind == W.KIND_ROT for g in c.gates)
    s = _rand_state(n, 50 + n)
    ref = s.copy()
    for g in c.gates:
        ref = _dense_gate(n, g, c.params) @ ref
    assert np.max(np.abs(O.run(c, state=s) - ref)) < 1e-13


# ------------------------------------------ multi-controlled gates (Sec. 2.4)
def _dense_controlled(n, controls, states, op):
    """P_c op + (I - P_c) with P_c the kron product of |v_q><v_q| on the
    control qubits (identity elsewhere)."""
    proj = [np.diag([1.0, 0.0]).astype(np.complex128), np.diag([0.0, 1.0]).astype(np.complex128)]
    f = [np.eye(2, dtype=np.complex128)] * n
    f = list(f)
    for c, v in zip(controls, states):
        f[c] = proj[v]
    P = kron_all(*f)
    return P @ op + (np.eye(2 ** n) - P)


def test_fig5_doubly_controlled_values():
    """Fig. 5: a doubly-controlled 1q gate on 3 qubits (controls q0 = q1 = 1,
    target q2) changes only the printed pair {6}, {7}, and that pair is U
    applied to (phi_6, phi_7)."""
    g = _gold("fig5_cc1q_n3.json")
    n = g["n"]
    rng = np.random.default_rng(70)
    u = W.haar_unitary(2, rng)
    phi = _rand_state(n, 71)
    c = W.Circuit(n, [W.with_controls(W.g1(g["target"], u), g["controls"])])
    out = O.run(c, state=phi)
    a, b = g["a"][0], g["b"][0]
    untouched = [x for x in range(2 ** n) if x not in (a, b)]
    assert np.array_equal(out[untouched], phi[untouched])
    assert np.max(np.abs(out[[a, b]] - u @ phi[[a, b]])) < 1e-15


@pytest.mark.parametrize("n", [3, 5, 6])
def test_controlled_gates_vs_dense_projector(n):
    """Extra controls on 1q, controlled-1q and 2q gates, any positions and
    control states, against the dense projector form built with kron."""
    rng = np.random.default_rng(72 + n)
    for trial in range(12):
        k = int(rng.integers(1, 3))             # gate qubits (1 or 2)
        nc = int(rng.integers(1, n - k + 1))    # extra controls
        qs = [int(x) for x in rng.choice(n, size=k + nc, replace=False)]
        tgt, ctrl = qs[:k], qs[k:]
        st = [int(x) for x in rng.integers(0, 2, size=nc)]
        phi = _rand_state(n, 80 + 10 * n + trial)
        if k == 1:
            u = W.haar_unitary(2, rng)
            gate, op = W.g1(tgt[0], u), dense_1q(n, tgt[0], u)
        elif trial % 2:
            u = W.haar_unitary(2, rng)
            cs = int(rng.integers(2))
            gate, op = W.gc(tgt[0], tgt[1], u, cs), dense_c1q(n, tgt[0], tgt[1], u, cs)
        else:
            u = W.haar_unitary(4, rng)
            gate, op = W.g2(tgt[0], tgt[1], u), dense_2q(n, tgt[0], tgt[1], u)
        c = W.Circuit(n, [W.with_controls(gate, ctrl, st)])
        ref = _dense_controlled(n, ctrl, st, op) @ phi
        assert np.max(np.abs(O.run(c, state=phi) - ref)) < 1e-14, (trial, qs, st)


def test_toffoli_truth_table_and_single_control():
    """The Toffoli gate permutes |110> and |111> (qubits c0, c1, t) and fixes
    every other basis state; one extra control on a 1q gate is the controlled
    gate of Sec. 2.2."""
    n = 3
    for x in range(8):
        out = O.run(W.Circuit(n, [W.toffoli(0, 1, 2)]), state=O.basis(n, x))
        y = x ^ 1 if (x >> 1) == 3 else x
        assert np.array_equal(out, O.basis(n, y))
    rng = np.random.default_rng(74)
    u = W.haar_unitary(2, rng)
    phi = _rand_state(5, 75)
    for cs in (0, 1):
        a = O.run(W.Circuit(5, [W.with_controls(W.g1(4, u), (1,), (cs,))]), state=phi)
        assert np.array_equal(a, O.apply_c1q(phi, 1, 4, u, cs))


# ------------------------------------------------ k-qubit gates (Sec. 2.4)
def _haar(d, rng):
    return W.haar_unitary(d, rng)


def test_kq_on_every_qubit_is_plain_matvec():
    """k = n on qubits (0, .., n-1): the local index is the whole index, so
    the gate is U @ phi."""
    rng = np.random.default_rng(301)
    for n in (1, 2, 3, 4):
        u = _haar(2 ** n, rng)
        phi = W.random_state(n, 302 + n)
        np.testing.assert_allclose(O.apply_kq(phi, list(range(n)), u), u @ phi, atol=1e-14)


def test_kq_permuted_qubits_is_axis_transpose():
    """k = n on a permutation of the qubits: U acts on the state tensor with
    its axes in that order (numpy transpose, then matvec, then back)."""
    rng = np.random.default_rng(311)
    n = 4
    for _ in range(5):
        perm = [int(x) for x in rng.permutation(n)]
        u = _haar(2 ** n, rng)
        phi = W.random_state(n, int(rng.integers(1 << 30)))
        t = phi.reshape((2,) * n).transpose(perm).reshape(-1)
        want = (u @ t).reshape((2,) * n).transpose(np.argsort(perm)).reshape(-1)
        np.testing.assert_allclose(O.apply_kq(phi, perm, u), want, atol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_kq_contiguous_is_kron(k):
    """Contiguous ascending qubits (q, .., q+k-1): eq. (1), (I (x) U (x) I) phi."""
    rng = np.random.default_rng(320 + k)
    n = 6
    for q in range(n - k + 1):
        u = _haar(2 ** k, rng)
        phi = W.random_state(n, 330 + q)
        m = np.kron(np.kron(np.eye(2 ** q), u), np.eye(2 ** (n - q - k)))
        np.testing.assert_allclose(O.apply_kq(phi, list(range(q, q + k)), u), m @ phi, atol=1e-14)


def test_kq_product_gate_equals_single_qubit_gates():
    """U = A (x) B (x) C on non-contiguous qubits (a, b, c) in that order is A
    on a, B on b and C on c."""
    rng = np.random.default_rng(341)
    n = 7
    for _ in range(4):
        a, b, c = (int(x) for x in rng.choice(n, size=3, replace=False))
        A, B, C = _haar(2, rng), _haar(2, rng), _haar(2, rng)
        phi = W.random_state(n, int(rng.integers(1 << 30)))
        want = O.apply_1q(O.apply_1q(O.apply_1q(phi, a, A), b, B), c, C)
        np.testing.assert_allclose(O.apply_kq(phi, [a, b, c], np.kron(np.kron(A, B), C)), want,
                                   atol=1e-14)


def test_kq_toffoli_matrix_equals_doubly_controlled_x():
    """The 8 x 8 Toffoli permutation on (c0, c1, t) equals X on t with two
    extra controls (the multi-controlled form of the same gate)."""
    n = 5
    tof = np.eye(8, dtype=complex)
    tof[[6, 7]] = tof[[7, 6]]
    phi = W.random_state(n, 351)
    for c0, c1, t in [(0, 1, 2), (4, 0, 2), (3, 1, 0)]:
        want = O.run(W.Circuit(n, [W.toffoli(c0, c1, t)]), phi)
        np.testing.assert_allclose(O.apply_kq(phi, [c0, c1, t], tof), want, atol=1e-15)
