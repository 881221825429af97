"""GPU parity of multi-controlled gates (Sec. 2.4, Fig. 5) and of general
k-qubit gates on any qubits (Sec. 2.4), through the C ABI, against the FP64
CPU oracle on the same seeded inputs.  complex128: max |d amp| <= 1e-12;
complex64: infidelity <= 1e-6."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def infidelity(a64, b128):
    ov = np.vdot(a64.astype(np.complex128), b128)
    return 1.0 - abs(ov) ** 2


def check(q, got, ref, dtype):
    if dtype == q.QSV_C128:
        assert np.max(np.abs(got - ref)) <= TOL128
    else:
        assert infidelity(got, ref) <= 1e-6


def run_gpu(q, ctx, n, dtype, phi, fn):
    st = q.State(ctx, n, dtype)
    st.from_numpy(phi.astype(np.complex128 if dtype == q.QSV_C128 else np.complex64))
    fn(st)
    out = st.to_numpy()
    st.free()
    return out


def test_fig5_doubly_controlled_pair(q, ctx):
    """Fig. 5: with controls q0 = q1 = 1 on 3 qubits, the gate on q2 mixes
    exactly amplitudes 6 and 7 and leaves the rest alone."""
    with open(os.path.join(GOLDEN, "fig5_cc1q_n3.json")) as f:
        fx = json.load(f)
    n = fx["n"]
    u = W.haar_unitary(2, np.random.default_rng(501))
    phi = W.random_state(n, 502)
    got = run_gpu(q, ctx, n, q.QSV_C128, phi, lambda st: st.applyMC1q(fx["controls"], fx["target"], u))
    a, b = fx["a"][0], fx["b"][0]
    want = phi.copy()
    want[a], want[b] = u[0, 0] * phi[a] + u[0, 1] * phi[b], u[1, 0] * phi[a] + u[1, 1] * phi[b]
    assert np.max(np.abs(got - want)) <= 1e-15


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 5, 9, 12])
def test_mc1q_every_control_count(q, ctx, n, dtype):
    """0..n-1 controls on random qubits and states, targets and controls
    below and above the 128-byte line, against the oracle's projector form."""
    dt = q.QSV_C128 if dtype == "c128" else q.QSV_C64
    rng = np.random.default_rng(510 + n)
    for nc in sorted({0, 1, 2, 3, n - 1} & set(range(n))):
        for _ in range(3):
            qs = [int(x) for x in rng.choice(n, size=nc + 1, replace=False)]
            t, cs = qs[0], qs[1:]
            vals = [int(v) for v in rng.integers(0, 2, size=nc)]
            u = W.haar_unitary(2, rng)
            phi = W.random_state(n, int(rng.integers(1 << 30)))
            ref = O.run(W.Circuit(n, [W.with_controls(W.g1(t, u), cs, vals)]), phi)
            got = run_gpu(q, ctx, n, dt, phi, lambda st: st.applyMC1q(cs, t, u, vals))
            check(q, got, ref, dt)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_toffoli_and_controlled_2q(q, ctx, dtype):
    """Toffolis (the swap kernel), a controlled 1q gate with extra controls and
    a 2-qubit gate with extra controls, one at a time through a circuit."""
    dt = q.QSV_C128 if dtype == "c128" else q.QSV_C64
    n = 11
    rng = np.random.default_rng(520)
    gates = [W.toffoli(0, 10, 5), W.toffoli(1, 2, 0), W.toffoli(9, 8, 10),
             W.with_controls(W.gc(3, 7, W.haar_unitary(2, rng), 0), [0, 10], [1, 0]),
             W.with_controls(W.g2(6, 1, W.haar_unitary(4, rng)), [2, 9, 4], [0, 1, 1]),
             W.with_controls(W.g2(10, 0, W.haar_unitary(4, rng)), [5])]
    for g in gates:
        phi = W.random_state(n, int(rng.integers(1 << 30)))
        ref = O.run(W.Circuit(n, [g]), phi)
        for flags in (0, q.FLAG_NO_FUSE):
            got = run_gpu(q, ctx, n, dt, phi, lambda st: st.apply_circuit([g], flags=flags))
            check(q, got, ref, dt)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,seed", [(10, 1), (13, 2), (16, 3)])
def test_multicontrol_circuits_fused_and_unfused(q, ctx, n, seed, dtype):
    """Circuits mixing fused gates with multi-controlled ones (each its own
    pass, ordered against everything else): fused and one kernel per gate."""
    dt = q.QSV_C128 if dtype == "c128" else q.QSV_C64
    c = W.random_multicontrol(n, 160, seed=530 + seed)
    phi = W.random_state(n, 540 + seed)
    ref = O.run(c, phi)
    for flags in (0, q.FLAG_NO_FUSE):
        got = run_gpu(q, ctx, n, dt, phi, lambda st: st.apply_circuit(c.gates, flags=flags))
        check(q, got, ref, dt)


def test_adjoint_through_multicontrolled_fixed_gates(q, ctx):
    """Gradients of a rotation ansatz interleaved with Toffolis and a
    multi-controlled Haar gate, fused and unfused, against the oracle's
    adjoint sweep."""
    n = 12
    base = W.hea_cz_ring(n, 3, seed=550)
    rng = np.random.default_rng(551)
    gates = []
    for k, g in enumerate(base.gates):
        gates.append(g)
        if k % 17 == 16:
            a, b, t = (int(x) for x in rng.choice(n, size=3, replace=False))
            gates.append(W.toffoli(a, b, t))
        if k % 29 == 28:
            t, c0, c1 = (int(x) for x in rng.choice(n, size=3, replace=False))
            gates.append(W.with_controls(W.g1(t, W.haar_unitary(2, rng)), [c0, c1], [1, 0]))
    c = W.Circuit(n, gates, base.params, base.observable)
    f_ref, g_ref = O.adjoint(c)
    sw = sum(abs(w) for _, w in c.observable)
    for flags in (q.FLAG_FORWARD, q.FLAG_FORWARD | q.FLAG_NO_FUSE):
        psi, lam = q.State(ctx, n, q.QSV_C128), q.State(ctx, n, q.QSV_C128)
        f, g = q.adjoint(psi, lam, c.gates, c.params, c.observable, flags=flags)
        psi.free()
        lam.free()
        assert abs(f - f_ref) <= 1e-12 * max(1.0, sw)
        assert np.max(np.abs(g - g_ref)) <= 1e-10 * max(1.0, sw)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_kq_any_qubits(q, ctx, k, dtype):
    """A Haar 2^k x 2^k gate on random qubits in random order (contiguous and
    not, below and above the 128-byte line) against the oracle."""
    dt = q.QSV_C128 if dtype == "c128" else q.QSV_C64
    rng = np.random.default_rng(560 + k)
    for n in sorted({k, k + 1, 9, 14}):
        for _ in range(2):
            qs = [int(x) for x in rng.choice(n, size=k, replace=False)]
            u = W.haar_unitary(2 ** k, rng)
            phi = W.random_state(n, int(rng.integers(1 << 30)))
            ref = O.apply_kq(phi, qs, u)
            got = run_gpu(q, ctx, n, dt, phi, lambda st: st.applyKq(qs, u))
            check(q, got, ref, dt)


def test_argument_errors_leave_state(q, ctx):
    n = 6
    phi = W.random_state(n, 570)
    st = q.State(ctx, n, q.QSV_C128)
    st.from_numpy(phi)
    u2 = np.eye(2)
    bad = [lambda: st.applyMC1q([1, 1], 0, u2),            # repeated control
           lambda: st.applyMC1q([0], 0, u2),               # control is the target
           lambda: st.applyMC1q([0, 1], 2, u2, [1, 2]),    # bad control state
           lambda: st.applyMC1q([7], 0, u2),               # out of range
           lambda: st.applyKq([0, 0], np.eye(4)),          # repeated qubit
           lambda: st.applyKq(list(range(6)), np.eye(64)),  # k > 5
           lambda: st.apply_circuit([W.with_controls(W.g1(0, u2), [0])]),   # control on own qubit
           lambda: st.apply_circuit([W.with_controls(W.g2(0, 1, np.eye(4)), [9])])]   # >= n
    for f in bad:
        with pytest.raises(q.QsvError):
            f()
    assert np.array_equal(st.to_numpy(), phi)
    st.free()
    with pytest.raises(q.QsvError):
        ctx.batch_run([W.Circuit(4, [W.toffoli(0, 1, 2)], np.zeros(0), [((0,), 1.0)])], q.QSV_C128)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qasm_program_through_the_library(q, ctx, dtype):
    """An OpenQASM 2.0 program (QFT on 12 qubits, then Toffoli, controlled
    swap and a user-defined gate) lowered by the front-end and run by
    qsv_apply_circuit, against the oracle on the same records and, for the
    QFT part, against numpy's FFT."""
    from paper_2303_00123_amd import qasm
    dt = q.QSV_C128 if dtype == "c128" else q.QSV_C64
    n = 12
    lines = ["OPENQASM 2.0;", 'include "qelib1.inc";', f"qreg q[{n}];"]
    for i in range(n):
        lines.append(f"h q[{i}];")
        for j in range(2, n - i + 1):
            lines.append(f"cu1(-2*pi/2^{j}) q[{j + i - 1}], q[{i}];")
    for i in range(n // 2):
        lines.append(f"swap q[{i}], q[{n - 1 - i}];")
    qft = qasm.parse("\n".join(lines))
    phi = W.random_state(n, 580)
    got = run_gpu(q, ctx, n, dt, phi, lambda st: st.apply_circuit(None, marshalled=qft.gates))
    check(q, got, np.fft.fft(phi) / np.sqrt(2 ** n), dt)
    tail = qasm.parse("\n".join(lines[:3] + [
        "gate g(a) x, y { ry(a) x; cz x, y; }", "ccx q[0], q[11], q[5];", "cswap q[3], q[1], q[10];",
        "g(0.3) q[2], q[7];", "c3x q[4], q[6], q[8], q[9];"]))
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import test_host_abi as H
    ref = O.run(H._records_to_circuit(n, tail.gates), phi)
    got = run_gpu(q, ctx, n, dt, phi, lambda st: st.apply_circuit(None, marshalled=tail.gates))
    check(q, got, ref, dt)
