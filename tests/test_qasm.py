"""OpenQASM 2.0 front-end (host logic): the parsed qsv_gate records, run by
the FP64 oracle, against independently built circuits, numpy FFT and dense
matrices; expression evaluation and error handling."""
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2303_00123_amd import qasm

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_host_abi import _records_to_circuit  # noqa: E402


def run(prog, phi):
    return O.run(_records_to_circuit(prog.n, prog.gates), phi)


def qft_qasm(n):
    lines = ["OPENQASM 2.0;", 'include "qelib1.inc";', f"qreg q[{n}];", f"creg c[{n}];"]
    for i in range(n):
        lines.append(f"h q[{i}];")
        for j in range(2, n - i + 1):
            lines.append(f"cu1(-2*pi/2^{j}) q[{j + i - 1}], q[{i}];")
    for i in range(n // 2):
        lines.append(f"swap q[{i}], q[{n - 1 - i}];")
    lines.append("measure q -> c;")
    return "\n".join(lines)


@pytest.mark.parametrize("n", [1, 3, 5, 8])
def test_qft_program_is_fft(n):
    """Fig. 1's QFT written in OpenQASM equals numpy.fft.fft(phi)/sqrt(N)."""
    prog = qasm.parse(qft_qasm(n))
    assert prog.n == n and len(prog.measures) == n
    phi = W.random_state(n, 700 + n)
    np.testing.assert_allclose(run(prog, phi), np.fft.fft(phi) / math.sqrt(2 ** n), atol=1e-13)


def test_gate_matrices_against_dense_definitions():
    """Each built-in gate on a 3-qubit register against its dense operator
    (numpy.kron of the textbook matrix, projector form for controls)."""
    n = 3
    X = np.array([[0, 1], [1, 0]], complex)
    Y = np.array([[0, -1j], [1j, 0]], complex)
    Z = np.diag([1, -1]).astype(complex)
    H = np.array([[1, 1], [1, -1]], complex) / math.sqrt(2)
    I2 = np.eye(2)

    def on(u, q):   # 1q operator on qubit q (qubit 0 = most significant)
        return np.kron(np.kron(np.eye(2 ** q), u), np.eye(2 ** (n - 1 - q)))

    def ctrl(u, c, t):
        P1 = np.diag([0, 1]).astype(complex)
        P0 = np.diag([1, 0]).astype(complex)
        a = [I2] * n
        b = [I2] * n
        a[c] = P0
        b[c] = P1
        b[t] = u
        k = lambda ms: np.kron(np.kron(ms[0], ms[1]), ms[2])
        return k(a) + k(b)

    def rot(P, t):
        return math.cos(t / 2) * np.eye(P.shape[0]) - 1j * math.sin(t / 2) * P

    th, ph, la = 0.7, -1.3, 2.1
    u3 = np.array([[math.cos(th / 2), -np.exp(1j * la) * math.sin(th / 2)],
                   [np.exp(1j * ph) * math.sin(th / 2), np.exp(1j * (ph + la)) * math.cos(th / 2)]])
    cases = {
        "x q[1];": on(X, 1), "y q[0];": on(Y, 0), "z q[2];": on(Z, 2), "h q[1];": on(H, 1),
        "s q[0];": on(np.diag([1, 1j]), 0), "tdg q[2];": on(np.diag([1, np.exp(-1j * math.pi / 4)]), 2),
        f"rx({th}) q[1];": on(rot(X, th), 1), f"ry({th}) q[2];": on(rot(Y, th), 2),
        f"rz({th}) q[0];": on(rot(Z, th), 0), f"u3({th},{ph},{la}) q[1];": on(u3, 1),
        f"u1({la}) q[2];": on(np.diag([1, np.exp(1j * la)]), 2),
        "cx q[0],q[2];": ctrl(X, 0, 2), "cz q[2],q[1];": ctrl(Z, 2, 1), "cy q[1],q[0];": ctrl(Y, 1, 0),
        "ch q[0],q[1];": ctrl(H, 0, 1), f"crz({th}) q[2],q[0];": ctrl(rot(Z, th), 2, 0),
        f"cu1({la}) q[1],q[2];": ctrl(np.diag([1, np.exp(1j * la)]), 1, 2),
        f"cu3({th},{ph},{la}) q[0],q[1];": ctrl(u3, 0, 1),
        "swap q[0],q[2];": ctrl(X, 0, 2) @ ctrl(X, 2, 0) @ ctrl(X, 0, 2),
        "ccx q[0],q[1],q[2];": np.eye(8)[[0, 1, 2, 3, 4, 5, 7, 6]],
        "ccx q[2],q[0],q[1];": np.eye(8)[[0, 1, 2, 3, 4, 7, 6, 5]],
        f"rzz({th}) q[0],q[2];": np.diag([np.exp(-1j * th / 2 * (1 - 2 * (((x >> 2) ^ x) & 1)))
                                         for x in range(8)]),
    }
    phi = W.random_state(n, 710)
    for stmt, M in cases.items():
        prog = qasm.parse(f"OPENQASM 2.0;\nqreg q[{n}];\n{stmt}")
        np.testing.assert_allclose(run(prog, phi), M @ phi, atol=1e-13, err_msg=stmt)


def test_cswap_and_c3x():
    n = 4
    phi = W.random_state(n, 720)
    prog = qasm.parse("OPENQASM 2.0; qreg a[2]; qreg b[2]; cswap a[1], b[0], a[0]; c3x b[1], a[0], a[1], b[0];")
    # qubits: a[0]=0, a[1]=1, b[0]=2, b[1]=3
    perm = np.arange(16)
    for x in range(16):   # cswap: control qubit 1, swap qubits 2 and 0
        b = [(x >> (3 - q)) & 1 for q in range(4)]
        if b[1]:
            b[2], b[0] = b[0], b[2]
        y = sum(v << (3 - q) for q, v in enumerate(b))
        perm[y] = x
    want = phi[perm]
    perm2 = np.arange(16)
    for x in range(16):   # c3x: controls 3, 0, 1; target 2
        b = [(x >> (3 - q)) & 1 for q in range(4)]
        if b[3] and b[0] and b[1]:
            b[2] ^= 1
        perm2[sum(v << (3 - q) for q, v in enumerate(b))] = x
    want = want[perm2]
    np.testing.assert_allclose(run(prog, phi), want, atol=1e-15)


def test_user_gates_broadcast_and_expressions():
    """A user-defined parametrised gate (expanded like a macro), register
    broadcasting and a parameter expression, against the same gates built
    with workloads."""
    text = """OPENQASM 2.0;
    include "qelib1.inc";
    // a two-qubit block with a parameter
    gate blk(a, b) x, y { ry(a/2) x; cx x, y; rz(-b*2 + sin(pi/6)) y; }
    qreg q[3]; qreg r[3];
    h q;
    blk(pi/3, 0.25) q, r;
    cx q[0], r;
    barrier q;
    """
    prog = qasm.parse(text)
    n = 6
    assert prog.n == n and prog.qregs == {"q": (0, 3), "r": (3, 3)}
    H = np.array([[1, 1], [1, -1]], complex) / math.sqrt(2)
    gates = [W.g1(i, H) for i in range(3)]
    a, b = math.pi / 3, 0.25
    for i in range(3):
        gates += [W.g1(i, O.rotation("Y", a / 2)), W.cnot(i, 3 + i),
                  W.g1(3 + i, O.rotation("Z", -b * 2 + math.sin(math.pi / 6)))]
    gates += [W.cnot(0, 3 + i) for i in range(3)]
    phi = W.random_state(n, 730)
    np.testing.assert_allclose(run(prog, phi), O.run(W.Circuit(n, gates), phi), atol=1e-14)


def test_expression_evaluator():
    env = {"t": 0.5}
    assert qasm.eval_expr("pi/2", {}) == math.pi / 2
    assert qasm.eval_expr("-2^3^2", {}) == -(2 ** 9)
    assert qasm.eval_expr("2*(t+1)-sqrt(4)/ln(exp(2))", env) == 2 * 1.5 - 1.0
    assert abs(qasm.eval_expr("cos(pi)+tan(0)+1e-3", {}) - (-1 + 1e-3)) < 1e-15
    for bad in ["pi/", "foo", "2 3", "sin(1"]:
        with pytest.raises(qasm.QasmError):
            qasm.eval_expr(bad, {})


@pytest.mark.parametrize("text", [
    "qreg q[2]; h q[2];",                 # index out of range
    "qreg q[2]; cx q[0], q[0];",          # repeated qubit
    "qreg q[2]; qreg p[3]; cx q, p;",     # register sizes differ
    "qreg q[2]; foo q[0];",               # unknown gate
    "qreg q[2]; rx q[0];",                # missing parameter
    "qreg q[2]; reset q[0];",             # unsupported statement
    "qreg q[2]; h q[0]",                  # unterminated
    "OPENQASM 3.0; qreg q[1];",           # version
])
def test_errors(text):
    with pytest.raises(qasm.QasmError):
        qasm.parse(text)
