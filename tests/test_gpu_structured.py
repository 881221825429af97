"""One-pass kernels for gates with structure (Sec. 2.1's X/Y/Z cases, the
CNOT of Sec. 2.2, the SWAP of Sec. 2.3, phase gates): diagonal gates touch
only the amplitudes they change, X/CNOT/SWAP only move data.  Each is
checked against the FP64 oracle through the C ABI's gate calls, one kernel
per gate in a circuit and the planner's single-gate pass, at low and high
index bits (below and above the 128-byte line) and both control states;
permutation gates must reproduce the oracle exactly."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

N = 14


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2303_00123_amd as qq
    return qq


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context()
    yield c
    c.close()


def phase(t):
    return W.phase(t)


S = phase(np.pi / 2)
T = phase(np.pi / 4)
RZ = np.diag([np.exp(-0.35j), np.exp(0.35j)])          # d0 != 1: every amplitude changes
ANTI = np.array([[0, np.exp(0.7j)], [np.exp(-1.1j), 0]])
ONE_Q = {"Z": (W.Z, "diag"), "S": (S, "diag"), "T": (T, "diag"), "P": (phase(1.234), "diag"),
         "RZ": (RZ, "diag"), "X": (W.X, "perm1q"), "Y": (W.Y, "anti1q"), "ANTI": (ANTI, "anti1q")}
CTRL = {"CZ": (W.Z, "diag"), "CP": (phase(-0.77), "diag"), "CRZ": (RZ, "diag"),
        "CNOT": (W.X, "cperm1q"), "CY": (W.Y, "canti1q")}
CNOT4 = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
CYC4 = np.array([[0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], dtype=complex)
TWO_Q = {"SWAP": (W.SWAP, "perm2q"), "CNOT4": (CNOT4, "perm2q"), "CYC4": (CYC4, "perm2q"),
         "CZ4": (np.diag([1, 1, 1, -1]).astype(complex), "diag"),
         "D4": (np.diag(np.exp(1j * np.array([0.1, -0.4, 0.9, 2.0]))), "diag")}
EXACT = {"perm1q", "cperm1q", "perm2q"}


def kernels_run(ctx, fn):
    ctx.profile_begin()
    fn()
    return set(ctx.profile_end())


def check(q, st, ref, kind, dt, base):
    got = st.to_numpy()
    if dt == q.QSV_C128:
        if kind in EXACT:
            assert np.array_equal(got, ref)
        else:
            assert np.max(np.abs(got - ref)) <= 1e-12
    else:
        if kind in EXACT:   # a permutation of the rounded input, exactly
            assert np.array_equal(got, ref.astype(np.complex64))
        else:
            assert np.max(np.abs(got.astype(np.complex128) - ref)) <= 1e-6


@pytest.mark.parametrize("dt_name", ["c128", "c64"])
def test_structured_1q(q, ctx, dt_name):
    dt = q.QSV_C128 if dt_name == "c128" else q.QSV_C64
    tag = "_" + dt_name
    phi = W.random_state(N, 61)
    if dt == q.QSV_C64:
        phi = phi.astype(np.complex64).astype(np.complex128)
    st = q.State(ctx, N, dt)
    for name, (u, kind) in ONE_Q.items():
        for qb in range(N):
            ref = O.apply_1q(phi, qb, u)
            st.from_numpy(phi)
            ran = kernels_run(ctx, lambda: st.apply1q(qb, u))
            assert kind + tag in ran, (name, qb, ran)
            check(q, st, ref, kind, dt, phi)
    st.free()


@pytest.mark.parametrize("dt_name", ["c128", "c64"])
def test_structured_controlled(q, ctx, dt_name):
    dt = q.QSV_C128 if dt_name == "c128" else q.QSV_C64
    tag = "_" + dt_name
    phi = W.random_state(N, 62)
    if dt == q.QSV_C64:
        phi = phi.astype(np.complex64).astype(np.complex128)
    st = q.State(ctx, N, dt)
    pairs = [(0, 1), (1, 0), (N - 1, 0), (0, N - 1), (N - 1, N - 2), (N - 2, N - 1), (5, 9), (N - 2, 3)]
    for name, (u, kind) in CTRL.items():
        for qc, qt in pairs:
            for cs in (0, 1):
                ref = O.apply_c1q(phi, qc, qt, u, cs)
                st.from_numpy(phi)
                ran = kernels_run(ctx, lambda: st.applyC1q(qc, qt, u, cs))
                assert kind + tag in ran, (name, qc, qt, cs, ran)
                check(q, st, ref, kind, dt, phi)
    st.free()


@pytest.mark.parametrize("dt_name", ["c128", "c64"])
def test_structured_2q(q, ctx, dt_name):
    dt = q.QSV_C128 if dt_name == "c128" else q.QSV_C64
    tag = "_" + dt_name
    phi = W.random_state(N, 63)
    if dt == q.QSV_C64:
        phi = phi.astype(np.complex64).astype(np.complex128)
    st = q.State(ctx, N, dt)
    pairs = [(0, 1), (1, 0), (N - 1, 0), (0, N - 1), (N - 1, N - 2), (N - 2, N - 1), (5, 9), (9, 5)]
    for name, (u, kind) in TWO_Q.items():
        for qa, qb in pairs:
            ref = O.apply_2q(phi, qa, qb, u)
            st.from_numpy(phi)
            ran = kernels_run(ctx, lambda: st.apply2q(qa, qb, u))
            assert kind + tag in ran, (name, qa, qb, ran)
            check(q, st, ref, kind, dt, phi)
    st.free()


def test_structured_gates_in_unfused_circuits_and_single_passes(q, ctx):
    """A circuit of structured gates applied one kernel per gate, and each
    gate alone through qsv_apply_circuit (a one-gate circuit is a single-gate
    pass of the planner), against the oracle; permutation-only circuits
    exactly."""
    rng = np.random.default_rng(64)
    gates = []
    for k in range(60):
        a, b = (int(x) for x in rng.choice(N, size=2, replace=False))
        r = k % 6
        if r == 0:
            gates.append(W.g1(a, [W.Z, S, T, RZ, W.X, W.Y][int(rng.integers(6))]))
        elif r == 1:
            gates.append(W.gc(a, b, [W.Z, phase(0.3), W.X, W.Y][int(rng.integers(4))], int(rng.integers(2))))
        elif r == 2:
            gates.append(W.g2(a, b, [W.SWAP, CNOT4, TWO_Q["D4"][0]][int(rng.integers(3))]))
        else:
            gates.append(W.g1(a, W.haar_unitary(2, rng)))
    c = W.Circuit(N, gates)
    phi = W.random_state(N, 65)
    ref = O.run(c, state=phi)
    st = q.State(ctx, N)
    st.from_numpy(phi)
    st.apply_circuit(c.gates, flags=q.FLAG_NO_FUSE)
    assert np.max(np.abs(st.to_numpy() - ref)) <= 1e-12
    v = phi.copy()
    st.from_numpy(phi)
    for g in c.gates:
        st.apply_circuit([g])
        v = O.run(W.Circuit(N, [g]), state=v)
    assert np.max(np.abs(st.to_numpy() - v)) <= 1e-12
    perm = [W.g1(3, W.X), W.gc(0, 7, W.X, 0), W.g2(2, 11, W.SWAP), W.gc(13, 1, W.X, 1),
            W.g2(12, 0, CYC4), W.g1(13, W.X)]
    cp = W.Circuit(N, perm)
    st.from_numpy(phi)
    st.apply_circuit(cp.gates, flags=q.FLAG_NO_FUSE)
    assert np.array_equal(st.to_numpy(), O.run(cp, state=phi))
    st.free()
