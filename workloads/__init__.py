"""Seeded synthetic circuit generators.

This module only *describes* circuits: which gate acts on which qubits, with
which explicit matrix or rotation angle.  It performs none of the simulation
arithmetic.  Both the FP64 CPU oracle (``oracle/``) and the HIP library
(``paper_2303_00123_amd``) consume these descriptions and marshal them into
their own structures, so the two sides see identical inputs.

Conventions
-----------
* Qubit ``q`` follows the paper's big-endian binary representation
  (Definition 1, Sec. 2): qubit 0 is the most significant bit of the
  amplitude index.
* A 2-qubit gate on ``(qa, qb)`` carries a 4x4 matrix in the local basis
  ``2*x_qa + x_qb`` -- the ordering eq. (1) gives for a contiguous pair with
  ``qa`` on the left.
* A controlled gate ``(qc, qt, cs)`` applies ``U`` to ``qt`` on the
  subspace where qubit ``qc`` equals ``cs`` (Sec. 2.2).
* A rotation ``("rot", q, axis, param)`` is ``exp(-i theta P / 2)`` with
  ``theta = params[param]`` and ``P`` the Pauli ``axis``.  Each side builds the
  2x2 matrix itself.

Haar-random unitaries follow Mezzadri's recipe (QR of a complex Ginibre
matrix with the phases of ``diag(R)`` divided out).  Random numbers come from
``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

KIND_1Q = "1q"
KIND_C1Q = "c1q"
KIND_2Q = "2q"
KIND_ROT = "rot"
AXES = ("X", "Y", "Z")


@dataclass(frozen=True)
class Gate:
    kind: str
    qubits: Tuple[int, ...]
    matrix: Optional[np.ndarray] = None   # complex128, 2x2 or 4x4
    ctrl_state: int = 1                   # c1q only
    axis: Optional[str] = None            # rot only
    param: int = -1                       # rot only: index into params
    # extra controls (Sec. 2.4): the gate acts only where each qubit in
    # `controls` holds the matching value in `control_states`
    controls: Tuple[int, ...] = ()
    control_states: Tuple[int, ...] = ()


@dataclass
class Circuit:
    n: int
    gates: List[Gate]
    params: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # observable: list of (tuple of qubits in the Z string, weight)
    observable: List[Tuple[Tuple[int, ...], float]] = field(default_factory=list)
    name: str = ""

    @property
    def num_gates(self) -> int:
        return len(self.gates)


# ---------------------------------------------------------------- matrices
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
I2 = np.eye(2, dtype=np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                dtype=np.complex128)


def phase(theta: float) -> np.ndarray:
    """P(theta) = diag(1, e^{i theta})."""
    return np.array([[1, 0], [0, np.exp(1j * theta)]], dtype=np.complex128)


def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed d x d unitary (Mezzadri 2007)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    dr = np.diag(r)
    return (q * (dr / np.abs(dr))[None, :]).astype(np.complex128)


# ----------------------------------------------------------- gate helpers
def g1(q: int, u: np.ndarray) -> Gate:
    return Gate(KIND_1Q, (int(q),), np.asarray(u, dtype=np.complex128))


def gc(qc: int, qt: int, u: np.ndarray, cs: int = 1) -> Gate:
    return Gate(KIND_C1Q, (int(qc), int(qt)), np.asarray(u, dtype=np.complex128), int(cs))


def g2(qa: int, qb: int, u: np.ndarray) -> Gate:
    return Gate(KIND_2Q, (int(qa), int(qb)), np.asarray(u, dtype=np.complex128))


def grot(q: int, axis: str, param: int) -> Gate:
    assert axis in AXES
    return Gate(KIND_ROT, (int(q),), None, 1, axis, int(param))


def with_controls(gate: Gate, controls: Sequence[int], states: Optional[Sequence[int]] = None) -> Gate:
    """The gate with extra control qubits (states default to 1): it then acts
    only where every one of them holds its state (a multi-controlled gate,
    Sec. 2.4)."""
    states = [1] * len(controls) if states is None else list(states)
    if len(states) != len(controls):
        raise ValueError("one state per control")
    return dataclasses.replace(gate, controls=tuple(int(c) for c in controls),
                               control_states=tuple(int(v) for v in states))


def toffoli(c0: int, c1: int, t: int) -> Gate:
    """Doubly-controlled X (Sec. 2.4): X on t where c0 = c1 = 1."""
    return with_controls(g1(t, X), (c0, c1))


def cnot(qc: int, qt: int) -> Gate:
    return gc(qc, qt, X, 1)


def cz(qa: int, qb: int) -> Gate:
    return gc(qa, qb, Z, 1)


# --------------------------------------------------------------- circuits
def random_mix(n: int, ngates: int, seed: int, name: str = "random_mix") -> Circuit:
    """50 % Haar 1q on a uniform qubit, 25 % controlled Haar 1q on a uniform
    ordered distinct (control, target) pair with control state 1, 25 % Haar 2q
    on a uniform ordered distinct pair.  Kinds drawn i.i.d. per gate."""
    if n < 2:
        raise ValueError("random_mix needs n >= 2")
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(ngates):
        r = rng.random()
        if r < 0.5:
            gates.append(g1(rng.integers(n), haar_unitary(2, rng)))
        elif r < 0.75:
            qc, qt = rng.choice(n, size=2, replace=False)
            gates.append(gc(qc, qt, haar_unitary(2, rng), 1))
        else:
            qa, qb = rng.choice(n, size=2, replace=False)
            gates.append(g2(qa, qb, haar_unitary(4, rng)))
    obs = [((q,), 1.0) for q in range(n)]
    return Circuit(n, gates, np.zeros(0), obs, name)


def random_multicontrol(n: int, ngates: int, seed: int, max_controls: int = 3,
                        name: str = "random_multicontrol") -> Circuit:
    """The 50/25/25 mix of `random_mix`, each gate given 0..max_controls extra
    controls (uniform count, on uniform distinct further qubits, each with a
    uniform control state), plus Toffolis (X with two controls in state 1)
    on every fifth gate.  Observable sum_i Z_i."""
    if n < 3:
        raise ValueError("random_multicontrol needs n >= 3")
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for k in range(ngates):
        if k % 5 == 4:
            c0, c1, t = rng.choice(n, size=3, replace=False)
            gates.append(toffoli(c0, c1, t))
            continue
        r = rng.random()
        if r < 0.5:
            g = g1(rng.integers(n), haar_unitary(2, rng))
        elif r < 0.75:
            qc, qt = rng.choice(n, size=2, replace=False)
            g = gc(qc, qt, haar_unitary(2, rng), int(rng.integers(2)))
        else:
            qa, qb = rng.choice(n, size=2, replace=False)
            g = g2(qa, qb, haar_unitary(4, rng))
        free = [q for q in range(n) if q not in g.qubits]
        nc = int(rng.integers(0, min(max_controls, len(free)) + 1))
        if nc:
            cs = rng.choice(free, size=nc, replace=False)
            g = with_controls(g, cs, rng.integers(0, 2, size=nc))
        gates.append(g)
    obs = [((q,), 1.0) for q in range(n)]
    return Circuit(n, gates, np.zeros(0), obs, f"{name}_n{n}_g{ngates}")


def mix_n10_g200(seed: int = 1001) -> Circuit:
    """10 qubits, 200 gates of the 50/25/25 mix; observables <Z_i> for all i."""
    return random_mix(10, 200, seed, "mix_n10_g200")


def layered_cnot_brick(n: int, layers: int, seed: int) -> Circuit:
    """Each layer: a Haar 1q gate on every qubit, then CNOTs on the even pairs
    (0,1),(2,3),... then on the odd pairs (1,2),(3,4),...  Control is the
    lower qubit number.  Observable Z_0 Z_{n-1}."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(layers):
        for q in range(n):
            gates.append(g1(q, haar_unitary(2, rng)))
        for q in range(0, n - 1, 2):
            gates.append(cnot(q, q + 1))
        for q in range(1, n - 1, 2):
            gates.append(cnot(q, q + 1))
    obs = [((0, n - 1), 1.0)]
    return Circuit(n, gates, np.zeros(0), obs, f"layered_cnot_brick_n{n}_l{layers}")


def brick_n28(n: int = 28, layers: int = 20, seed: int = 1002) -> Circuit:
    return layered_cnot_brick(n, layers, seed)


def layered_haar_pairs(n: int, layers: int, seed: int) -> Circuit:
    """Each layer: a Haar 1q gate on every qubit, then Haar 2q gates on the
    disjoint pairs of a fresh random permutation of the qubits (consecutive
    entries paired).  Observable sum_i Z_i."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(layers):
        for q in range(n):
            gates.append(g1(q, haar_unitary(2, rng)))
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            gates.append(g2(perm[i], perm[i + 1], haar_unitary(4, rng)))
    obs = [((q,), 1.0) for q in range(n)]
    return Circuit(n, gates, np.zeros(0), obs, f"layered_haar_pairs_n{n}_l{layers}")


def haar_pairs_n32(n: int = 32, layers: int = 10, seed: int = 1003) -> Circuit:
    return layered_haar_pairs(n, layers, seed)


def ry_rz_cnot_ladder(n: int, layers: int, rng: np.random.Generator,
                      name: str = "ry_rz_ladder") -> Circuit:
    """Each layer: RY(theta) then RZ(phi) on every qubit (time order), then a
    CNOT ladder (0,1),(1,2),...,(n-2,n-1).  Angles uniform in [0, 2 pi).
    Observable sum_i Z_i."""
    gates: List[Gate] = []
    params: List[float] = []
    for _ in range(layers):
        for q in range(n):
            gates.append(grot(q, "Y", len(params)))
            params.append(rng.uniform(0.0, 2.0 * np.pi))
            gates.append(grot(q, "Z", len(params)))
            params.append(rng.uniform(0.0, 2.0 * np.pi))
        for q in range(n - 1):
            gates.append(cnot(q, q + 1))
    obs = [((q,), 1.0) for q in range(n)]
    return Circuit(n, gates, np.asarray(params, dtype=np.float64), obs, name)


def ladder_batch_256(nb: int = 256, layers: int = 6, nmin: int = 12, nmax: int = 20,
            seed_base: int = 4000) -> List[Circuit]:
    """Batch of parametrised circuits; circuit b draws its qubit count and
    angles from default_rng(seed_base + b)."""
    out = []
    for b in range(nb):
        rng = np.random.default_rng(seed_base + b)
        n = int(rng.integers(nmin, nmax + 1))
        out.append(ry_rz_cnot_ladder(n, layers, rng, f"batch{b}_n{n}"))
    return out


def hea_cz_ring(n: int, layers: int, seed: int, ring_obs: bool = False) -> Circuit:
    """Hardware-efficient ansatz: per layer RY then RZ on every qubit, then a
    CZ ring (i, i+1 mod n) for i = 0..n-1.  Angles uniform in [0, 2 pi).
    Observable sum_i w_i Z_i Z_{i+1}, w_i ~ N(0,1), open chain i = 0..n-2
    (ring closes it with (n-1, 0))."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    params: List[float] = []
    for _ in range(layers):
        for q in range(n):
            gates.append(grot(q, "Y", len(params)))
            params.append(rng.uniform(0.0, 2.0 * np.pi))
            gates.append(grot(q, "Z", len(params)))
            params.append(rng.uniform(0.0, 2.0 * np.pi))
        if n >= 2:
            for q in range(n):
                a, b = q, (q + 1) % n
                if n == 2 and q == 1:
                    break
                gates.append(cz(a, b))
    nterm = n if (ring_obs and n > 2) else n - 1
    w = rng.standard_normal(nterm)
    obs = [((i, (i + 1) % n), float(w[i])) for i in range(nterm)]
    return Circuit(n, gates, np.asarray(params, dtype=np.float64), obs,
                   f"hea_cz_ring_n{n}_l{layers}")


def hea_n24(n: int = 24, layers: int = 10, seed: int = 1005) -> Circuit:
    return hea_cz_ring(n, layers, seed)


def mixed_param_circuit(n: int, layers: int, seed: int) -> Circuit:
    """Rotations interleaved with fixed gates that are not their own inverse,
    for gradient checks through general gates.  Each layer: a rotation on
    every qubit (axis X, Y, Z in turn), a Haar 1q gate on a random qubit,
    Haar 2q gates on a random pair in ascending and in descending qubit
    order, controlled Haar gates with control state 0 and 1 on random
    ordered pairs, then one more rotation.  Every parameter drives one
    rotation.  Observable: sum_i w_i Z_i Z_{i+1} plus w_n Z_0, w ~ N(0, 1)."""
    if n < 2:
        raise ValueError("mixed_param_circuit needs n >= 2")
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    params: List[float] = []

    def rot(q: int, axis: str):
        gates.append(grot(q, axis, len(params)))
        params.append(rng.uniform(0.0, 2.0 * np.pi))

    for layer in range(layers):
        for q in range(n):
            rot(q, AXES[(q + layer) % 3])
        gates.append(g1(int(rng.integers(n)), haar_unitary(2, rng)))
        a, b = sorted(int(x) for x in rng.choice(n, size=2, replace=False))
        gates.append(g2(a, b, haar_unitary(4, rng)))
        a, b = sorted(int(x) for x in rng.choice(n, size=2, replace=False))
        gates.append(g2(b, a, haar_unitary(4, rng)))
        for cs in (0, 1):
            qc, qt = (int(x) for x in rng.choice(n, size=2, replace=False))
            gates.append(gc(qc, qt, haar_unitary(2, rng), cs))
        rot(int(rng.integers(n)), AXES[layer % 3])
    w = rng.standard_normal(n)
    obs = [((i, i + 1), float(w[i])) for i in range(n - 1)] + [((0,), float(w[n - 1]))]
    return Circuit(n, gates, np.asarray(params, dtype=np.float64), obs,
                   f"mixed_param_n{n}_l{layers}")


def trotter_tfxy(n: int, steps: int, seed: int) -> Circuit:
    """Trotter time-evolution circuit of a 1D nearest-neighbour TFXY chain,
    with the structure of the paper's Hamiltonian-simulation benchmark:
    per step an RZ on every qubit, then on each even pair (q, q+1) the block
    CNOT(q, q+1) . (RX on q, RZ on q+1) . CNOT(q, q+1), an RZ on every qubit,
    the same blocks on the odd pairs; after the last step an RZ on every
    qubit the odd blocks touch.  The paper gives neither the angles nor the
    number of steps: angles are drawn uniform in [0, 2 pi) (one parameter per
    rotation).  No observable."""
    if n < 2:
        raise ValueError("trotter_tfxy needs n >= 2")
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    params: List[float] = []

    def rot(q: int, axis: str):
        gates.append(grot(q, axis, len(params)))
        params.append(rng.uniform(0.0, 2.0 * np.pi))

    def blocks(first: int):
        for q in range(first, n - 1, 2):
            gates.append(cnot(q, q + 1))
            rot(q, "X")
            rot(q + 1, "Z")
            gates.append(cnot(q, q + 1))

    for _ in range(steps):
        for q in range(n):
            rot(q, "Z")
        blocks(0)
        for q in range(n):
            rot(q, "Z")
        blocks(1)
    for q in range(1, 2 * ((n - 1) // 2) + 1):
        rot(q, "Z")
    return Circuit(n, gates, np.asarray(params, dtype=np.float64), [],
                   f"trotter_tfxy_n{n}_s{steps}")


def qft(n: int) -> Circuit:
    """QFT circuit as printed in Fig. 1 of the paper: for each i, H(i) then
    controlled-phase CP(ctrl=j+i-1, tgt=i, theta=-2 pi / 2^j) for j=2..n-i;
    then SWAP(i, n-1-i) for i < floor(n/2)."""
    gates: List[Gate] = []
    for i in range(n):
        gates.append(g1(i, H))
        for j in range(2, n - i + 1):
            gates.append(gc(j + i - 1, i, phase(-2.0 * np.pi / (2 ** j)), 1))
    for i in range(n // 2):
        gates.append(g2(i, n - i - 1, SWAP))
    return Circuit(n, gates, np.zeros(0), [], f"qft_n{n}")


def inverse(c: Circuit) -> Circuit:
    """The inverse circuit: gates reversed, each replaced by its adjoint.
    Rotations get a negated angle through a fresh parameter vector."""
    gates: List[Gate] = []
    params = list(-np.asarray(c.params, dtype=np.float64))
    for g in reversed(c.gates):
        if g.kind == KIND_ROT:
            gates.append(g)
        else:
            gates.append(dataclasses.replace(g, matrix=g.matrix.conj().T.copy()))
    return Circuit(c.n, gates, np.asarray(params, dtype=np.float64), [], c.name + "_inv")


def random_state(n: int, seed: int) -> np.ndarray:
    """Normalised complex Gaussian state of 2^n amplitudes."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    return (v / np.linalg.norm(v)).astype(np.complex128)


def observable_masks(obs: Sequence[Tuple[Tuple[int, ...], float]]):
    """(qubit bit masks: bit q set for qubit q in the Z string, weights)."""
    masks = np.array([sum(1 << q for q in qs) for qs, _ in obs], dtype=np.uint64)
    w = np.array([wt for _, wt in obs], dtype=np.float64)
    return masks, w
