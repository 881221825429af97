"""FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The GPU library neither imports nor links
anything here, and nothing here imports the GPU library.

The arithmetic lives in ``qsv_oracle.c`` (plain C, FP64, gates applied by
their Kronecker-product definition, eq. (1) of Sec. 2).  This module compiles
it with the host C compiler and marshals ``workloads.Circuit`` descriptions
into the C gate records.  ``indices.py`` holds the paper's index maps
(Algs. 1-3) as enumerations, for checking pairings against Figs. 3-5.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_1Q, ORC_C1Q, ORC_2Q, ORC_ROT = 0, 1, 2, 3
_KIND = {W.KIND_1Q: ORC_1Q, W.KIND_C1Q: ORC_C1Q, W.KIND_2Q: ORC_2Q, W.KIND_ROT: ORC_ROT}
_AXIS = {"X": 0, "Y": 1, "Z": 2}

GATE_DTYPE = np.dtype([("kind", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("cs", "<i4"),
                       ("axis", "<i4"), ("param", "<i4"), ("m", "<f8", (32,)),
                       ("cmask", "<u8"), ("cvals", "<u8")], align=True)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        i, i64, u64, d = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.orc_apply_1q.argtypes = [i, vp, vp, i, vp]
        L.orc_apply_c1q.argtypes = [i, vp, vp, i, i, i, vp]
        L.orc_apply_2q.argtypes = [i, vp, vp, i, i, vp]
        L.orc_apply_kq.argtypes = [i, vp, vp, i, vp, vp]
        L.orc_rotation.argtypes = [i, d, vp]
        L.orc_run.argtypes = [i, vp, vp, i64, vp, vp]
        L.orc_init_basis.argtypes = [i, vp, u64]
        L.orc_norm2.argtypes = [i, vp]
        L.orc_norm2.restype = d
        L.orc_expect_z.argtypes = [i, vp, u64]
        L.orc_expect_z.restype = d
        L.orc_inner.argtypes = [i, vp, vp, vp]
        L.orc_prob1.argtypes = [i, vp, i]
        L.orc_prob1.restype = d
        L.orc_measure1.argtypes = [i, vp, i, d]
        L.orc_measure1.restype = i
        L.orc_expect_obs.argtypes = [i, vp, i, vp, vp]
        L.orc_expect_obs.restype = d
        L.orc_energy.argtypes = [i, i64, vp, vp, i, vp, vp, vp, vp]
        L.orc_energy.restype = d
        L.orc_adjoint.argtypes = [i, i64, vp, vp, i, i, vp, vp, vp, vp, vp, vp]
        L.orc_adjoint.restype = d
        L.orc_param_shift.argtypes = [i, i64, vp, vp, i, i, vp, i, vp, vp, vp, vp, vp]
        L.orc_finite_diff.argtypes = [i, i64, vp, vp, i, i, vp, d, i, vp, vp, vp, vp, vp]
        L.orc_product_amplitude.argtypes = [i, vp, u64, vp]
        L.orc_num_threads.restype = i
        L.orc_set_num_threads.argtypes = [i]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _mat(u: np.ndarray) -> np.ndarray:
    u = _c128(u)
    return np.ascontiguousarray(np.stack([u.real, u.imag], axis=-1).reshape(-1))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int) -> None:
    lib().orc_set_num_threads(int(t))


# ------------------------------------------------------------ single gates
def apply_1q(state: np.ndarray, q: int, u: np.ndarray) -> np.ndarray:
    s = _c128(state)
    n = int(np.log2(s.size))
    out = np.empty_like(s)
    lib().orc_apply_1q(n, _p(s), _p(out), q, _p(_mat(u)))
    return out


def apply_c1q(state: np.ndarray, qc: int, qt: int, u: np.ndarray, cs: int = 1) -> np.ndarray:
    s = _c128(state)
    n = int(np.log2(s.size))
    out = np.empty_like(s)
    lib().orc_apply_c1q(n, _p(s), _p(out), qc, qt, cs, _p(_mat(u)))
    return out


def apply_2q(state: np.ndarray, qa: int, qb: int, u: np.ndarray) -> np.ndarray:
    s = _c128(state)
    n = int(np.log2(s.size))
    out = np.empty_like(s)
    lib().orc_apply_2q(n, _p(s), _p(out), qa, qb, _p(_mat(u)))
    return out


def apply_kq(state: np.ndarray, qubits: Sequence[int], u: np.ndarray) -> np.ndarray:
    """A 2^k x 2^k gate on `qubits` (qubits[0] = most significant local bit)."""
    s = _c128(state)
    n = int(np.log2(s.size))
    qs = np.ascontiguousarray(list(qubits), dtype=np.int32)
    out = np.empty_like(s)
    lib().orc_apply_kq(n, _p(s), _p(out), int(qs.size), _p(qs), _p(_mat(u)))
    return out


def rotation(axis: str, theta: float) -> np.ndarray:
    u = np.zeros(8)
    lib().orc_rotation(_AXIS[axis], float(theta), _p(u))
    return (u[0::2] + 1j * u[1::2]).reshape(2, 2)


# ---------------------------------------------------------------- circuits
def marshal(circ: W.Circuit) -> np.ndarray:
    g = np.zeros(len(circ.gates), dtype=GATE_DTYPE)
    for k, gate in enumerate(circ.gates):
        g["kind"][k] = _KIND[gate.kind]
        g["param"][k] = -1
        if gate.kind == W.KIND_ROT:
            g["q0"][k] = gate.qubits[0]
            g["axis"][k] = _AXIS[gate.axis]
            g["param"][k] = gate.param
        else:
            g["q0"][k] = gate.qubits[0]
            if len(gate.qubits) > 1:
                g["q1"][k] = gate.qubits[1]
            g["cs"][k] = gate.ctrl_state
            m = _mat(gate.matrix)
            g["m"][k][: m.size] = m
        for q, v in zip(gate.controls, gate.control_states):
            g["cmask"][k] |= np.uint64(1 << int(q))
            if v:
                g["cvals"][k] |= np.uint64(1 << int(q))
    return g


def run(circ: W.Circuit, state: Optional[np.ndarray] = None, ngates: Optional[int] = None) -> np.ndarray:
    """Final state of the circuit applied to ``state`` (default |0...0>)."""
    n = circ.n
    if state is None:
        s = np.zeros(2 ** n, dtype=np.complex128)
        s[0] = 1.0
    else:
        s = _c128(state).copy()
    work = np.empty_like(s)
    g = marshal(circ)
    ng = len(circ.gates) if ngates is None else int(ngates)
    params = np.ascontiguousarray(circ.params, dtype=np.float64)
    if params.size == 0:
        params = np.zeros(1)
    lib().orc_run(n, _p(s), _p(work), ng, _p(g), _p(params))
    return s


def basis(n: int, b: int = 0) -> np.ndarray:
    s = np.empty(2 ** n, dtype=np.complex128)
    lib().orc_init_basis(n, _p(s), b)
    return s


# ---------------------------------------------------------------- reductions
def norm2(state: np.ndarray) -> float:
    s = _c128(state)
    return float(lib().orc_norm2(int(np.log2(s.size)), _p(s)))


def expect_z(state: np.ndarray, qubits: Sequence[int]) -> float:
    s = _c128(state)
    mask = sum(1 << int(q) for q in qubits)
    return float(lib().orc_expect_z(int(np.log2(s.size)), _p(s), mask))


def expect_obs(state: np.ndarray, obs) -> float:
    s = _c128(state)
    masks, w = W.observable_masks(obs)
    return float(lib().orc_expect_obs(int(np.log2(s.size)), _p(s), len(w), _p(masks), _p(w)))


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    a = _c128(a)
    b = _c128(b)
    out = np.zeros(2)
    lib().orc_inner(int(np.log2(a.size)), _p(a), _p(b), _p(out))
    return complex(out[0], out[1])


def prob1(state: np.ndarray, q: int) -> float:
    s = _c128(state)
    return float(lib().orc_prob1(int(np.log2(s.size)), _p(s), q))


def measure1(state: np.ndarray, q: int, r: float):
    """Returns (outcome, collapsed state)."""
    s = _c128(state).copy()
    k = int(lib().orc_measure1(int(np.log2(s.size)), _p(s), q, float(r)))
    return k, s


def product_amplitude(qstates: np.ndarray, x: int) -> complex:
    """<x| (q_0 (x) q_1 (x) ... ) for per-qubit 2-vectors qstates[q]."""
    qs = _c128(qstates)
    n = qs.shape[0]
    flat = np.ascontiguousarray(np.stack([qs.real, qs.imag], axis=-1).reshape(-1))
    out = np.zeros(2)
    lib().orc_product_amplitude(n, _p(flat), int(x), _p(out))
    return complex(out[0], out[1])


# ------------------------------------------------------------- gradients
def _obs_args(circ: W.Circuit):
    masks, w = W.observable_masks(circ.observable)
    return masks, w


def energy(circ: W.Circuit, params: Optional[np.ndarray] = None) -> float:
    n = circ.n
    g = marshal(circ)
    p = np.ascontiguousarray(circ.params if params is None else params, dtype=np.float64)
    if p.size == 0:
        p = np.zeros(1)
    masks, w = _obs_args(circ)
    s = np.empty(2 ** n, dtype=np.complex128)
    work = np.empty_like(s)
    return float(lib().orc_energy(n, len(g), _p(g), _p(p), len(w), _p(masks), _p(w), _p(s), _p(work)))


def adjoint(circ: W.Circuit):
    """(f, grad) by the adjoint method."""
    n = circ.n
    g = marshal(circ)
    p = np.ascontiguousarray(circ.params, dtype=np.float64)
    npar = p.size
    if p.size == 0:
        p = np.zeros(1)
    masks, w = _obs_args(circ)
    grad = np.zeros(max(npar, 1))
    bufs = [np.empty(2 ** n, dtype=np.complex128) for _ in range(3)]
    f = lib().orc_adjoint(n, len(g), _p(g), _p(p), npar, len(w), _p(masks), _p(w), _p(grad),
                          *[_p(b) for b in bufs])
    return float(f), grad[:npar]


def param_shift(circ: W.Circuit, sel: Optional[Sequence[int]] = None) -> np.ndarray:
    n = circ.n
    g = marshal(circ)
    p = np.ascontiguousarray(circ.params, dtype=np.float64)
    sel = np.arange(p.size, dtype=np.int32) if sel is None else np.asarray(sel, dtype=np.int32)
    masks, w = _obs_args(circ)
    out = np.zeros(max(sel.size, 1))
    s = np.empty(2 ** n, dtype=np.complex128)
    work = np.empty_like(s)
    lib().orc_param_shift(n, len(g), _p(g), _p(p), p.size, sel.size, _p(sel), len(w), _p(masks),
                          _p(w), _p(out), _p(s), _p(work))
    return out[: sel.size]


def finite_diff(circ: W.Circuit, sel: Optional[Sequence[int]] = None, h: float = 1e-6) -> np.ndarray:
    n = circ.n
    g = marshal(circ)
    p = np.ascontiguousarray(circ.params, dtype=np.float64)
    sel = np.arange(p.size, dtype=np.int32) if sel is None else np.asarray(sel, dtype=np.int32)
    masks, w = _obs_args(circ)
    out = np.zeros(max(sel.size, 1))
    s = np.empty(2 ** n, dtype=np.complex128)
    work = np.empty_like(s)
    lib().orc_finite_diff(n, len(g), _p(g), _p(p), p.size, sel.size, _p(sel), float(h), len(w),
                          _p(masks), _p(w), _p(out), _p(s), _p(work))
    return out[: sel.size]
