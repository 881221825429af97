"""ctypes binding of libqsv.so (include/qsv.h).

Argument marshalling only: every step of the simulation runs in the HIP
library.  PyTorch supplies device memory (state tensors) and the HIP stream.
If the library has not been built this module raises on first use; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsv.so")

QSV_OK = 0
QSV_C64, QSV_C128 = 1, 2
G1Q, GC1Q, G2Q, GROT = 0, 1, 2, 3
FLAG_NO_FUSE, FLAG_FORWARD, FLAG_CAPTURE_GRAPH, FLAG_TUNE, FLAG_FROM_ZERO = 1, 2, 4, 8, 16
AXES = {"X": 0, "Y": 1, "Z": 2}
KINDS = {"1q": G1Q, "c1q": GC1Q, "2q": G2Q, "rot": GROT}

STATUS = {0: "QSV_OK", 1: "QSV_ERR_ARG", 2: "QSV_ERR_QUBIT", 3: "QSV_ERR_NOMEM",
          4: "QSV_ERR_HIP", 5: "QSV_ERR_DTYPE", 6: "QSV_ERR_ALIGN", 7: "QSV_ERR_SIZE",
          8: "QSV_ERR_INTERNAL"}

# C layout of qsv_gate: 6 x int32, double[32] (offset 24), then the extra
# control masks cmask, cvals (uint64 at 280, 288): 296 bytes.
GATE_DTYPE = np.dtype([("kind", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("ctrl_state", "<i4"),
                       ("axis", "<i4"), ("param", "<i4"), ("m", "<f8", (32,)),
                       ("cmask", "<u8"), ("cvals", "<u8")], align=True)
assert GATE_DTYPE.itemsize == 296


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


# every symbol the header declares
EXPORTS = [
    "qsv_ctx_create", "qsv_ctx_set_stream", "qsv_ctx_destroy", "qsv_sync", "qsv_status_str",
    "qsv_last_error", "qsv_state_wrap", "qsv_state_alloc", "qsv_state_free", "qsv_state_info",
    "qsv_init_basis", "qsv_apply1q", "qsv_applyC1q", "qsv_apply2q", "qsv_apply_circuit",
    "qsv_norm2", "qsv_expect_z", "qsv_inner", "qsv_prob1", "qsv_measure1", "qsv_copy_to_host",
    "qsv_copy_from_host", "qsv_adjoint", "qsv_batch_run", "qsv_profile_begin", "qsv_profile_end",
    "qsv_set_tile", "qsv_plan_circuit", "qsv_plan_fused", "qsv_applyMC1q", "qsv_applyKq",
    "qsv_expect_z_dev", "qsv_set_jit", "qsv_jit_stats", "qsv_jit_source", "qsv_set_matrix_cores",
]


class QsvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libqsv.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python -m paper_2303_00123_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, d, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                ctypes.c_double, ctypes.c_size_t)
    P = ctypes.POINTER
    sig = {
        "qsv_ctx_create": [vp, P(vp)],
        "qsv_ctx_set_stream": [vp, vp],
        "qsv_ctx_destroy": [vp],
        "qsv_sync": [vp],
        "qsv_state_wrap": [vp, vp, sz, i32, i32, P(vp)],
        "qsv_state_alloc": [vp, i32, i32, P(vp)],
        "qsv_state_free": [vp],
        "qsv_state_info": [vp, P(i32), P(i32), P(vp)],
        "qsv_init_basis": [vp, u64],
        "qsv_apply1q": [vp, i32, vp],
        "qsv_applyC1q": [vp, i32, i32, i32, vp],
        "qsv_apply2q": [vp, i32, i32, vp],
        "qsv_applyMC1q": [vp, i32, vp, vp, i32, vp],
        "qsv_applyKq": [vp, i32, vp, vp],
        "qsv_apply_circuit": [vp, vp, i64, vp, i64, i32],
        "qsv_norm2": [vp, P(d)],
        "qsv_expect_z": [vp, i32, vp, vp, vp, vp],
        "qsv_expect_z_dev": [vp, i32, vp, vp],
        "qsv_set_jit": [vp, i32],
        "qsv_set_matrix_cores": [vp, i32],
        "qsv_jit_stats": [vp, P(i32), P(d)],
        "qsv_jit_source": [i32, i32, vp, i64, vp, i64, i64, vp, sz, P(sz)],
        "qsv_inner": [vp, vp, vp],
        "qsv_prob1": [vp, i32, P(d)],
        "qsv_measure1": [vp, i32, d, P(i32)],
        "qsv_copy_to_host": [vp, vp, sz],
        "qsv_copy_from_host": [vp, vp, sz],
        "qsv_adjoint": [vp, vp, vp, i64, vp, i64, i32, vp, vp, vp, vp, i32],
        "qsv_batch_run": [vp, i32, vp, vp, vp, vp, i64, vp, vp, vp, i32, vp, i32],
        "qsv_profile_begin": [vp],
        "qsv_profile_end": [vp, vp, i32, P(i32)],
        "qsv_set_tile": [vp, i32, i32, i32, i32, i32],
        "qsv_plan_circuit": [i32, i32, vp, i64, i32, i32, i32, P(i64), vp, vp, vp],
        "qsv_plan_fused": [i32, i32, vp, i64, vp, i64, i32, i32, i32, i32, vp, i64, vp, P(i64)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    L.qsv_status_str.argtypes = [ctypes.c_int32]
    L.qsv_status_str.restype = ctypes.c_char_p
    L.qsv_last_error.argtypes = [vp]
    L.qsv_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _mat(u, dim: int) -> np.ndarray:
    u = np.asarray(u, dtype=np.complex128).reshape(dim, dim)
    return np.ascontiguousarray(np.stack([u.real, u.imag], axis=-1).reshape(-1))


def marshal_gates(gates: Iterable) -> np.ndarray:
    """Gate objects (attributes kind, qubits, matrix, ctrl_state, axis, param)
    -> array of qsv_gate records."""
    gates = list(gates)
    g = np.zeros(len(gates), dtype=GATE_DTYPE)
    for i, gate in enumerate(gates):
        kind = KINDS[gate.kind]
        g["kind"][i] = kind
        g["q0"][i] = gate.qubits[0]
        g["param"][i] = -1
        if len(gate.qubits) > 1:
            g["q1"][i] = gate.qubits[1]
        if kind == GROT:
            g["axis"][i] = AXES[gate.axis]
            g["param"][i] = gate.param
        else:
            g["ctrl_state"][i] = getattr(gate, "ctrl_state", 1)
            m = _mat(gate.matrix, 4 if kind == G2Q else 2)
            g["m"][i][: m.size] = m
        for q, v in zip(getattr(gate, "controls", ()), getattr(gate, "control_states", ())):
            g["cmask"][i] |= np.uint64(1 << int(q))
            if v:
                g["cvals"][i] |= np.uint64(1 << int(q))
    return g


def observable_arrays(obs) -> tuple:
    """[(qubits, weight), ...] -> (uint64 qubit masks, float64 weights)."""
    masks = np.array([sum(1 << int(q) for q in qs) for qs, _ in obs], dtype=np.uint64)
    w = np.array([float(wt) for _, wt in obs], dtype=np.float64)
    return masks, w


def _torch():
    import torch
    return torch


class Context:
    """A qsv_ctx bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, stream: Optional[int] = None):
        L = lib()
        if stream is None:
            torch = _torch()
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = ctypes.c_void_p()
        st = L.qsv_ctx_create(ctypes.c_void_p(stream), ctypes.byref(h))
        if st != QSV_OK:
            raise QsvError(st, "qsv_ctx_create failed")
        self.handle = h

    def check(self, st: int):
        if st != QSV_OK:
            raise QsvError(st, lib().qsv_last_error(self.handle).decode())

    def set_stream(self, stream: int):
        self.check(lib().qsv_ctx_set_stream(self.handle, ctypes.c_void_p(stream)))
        self._stream = stream

    def sync(self):
        self.check(lib().qsv_sync(self.handle))

    def set_tile(self, dtype: int, tile_bits: int = 0, low_bits: int = 0, reg_bits: int = 0,
                 lds_rounds: int = 0):
        self.check(lib().qsv_set_tile(self.handle, dtype, tile_bits, low_bits, reg_bits, lds_rounds))

    def set_jit(self, mode: int):
        self.check(lib().qsv_set_jit(self.handle, mode))

    def set_matrix_cores(self, mode: int):
        """Dense k-qubit gates on the MFMA units: 1 (default) for k = 3 and 5,
        2 for every k in 3..5, 0 never (vector units)."""
        self.check(lib().qsv_set_matrix_cores(self.handle, mode))

    def jit_stats(self) -> tuple:
        k, t = ctypes.c_int(), ctypes.c_double()
        self.check(lib().qsv_jit_stats(self.handle, ctypes.byref(k), ctypes.byref(t)))
        return k.value, t.value

    def profile_begin(self):
        self.check(lib().qsv_profile_begin(self.handle))

    def profile_end(self) -> dict:
        arr = (KStat * 64)()
        cnt = ctypes.c_int()
        self.check(lib().qsv_profile_end(self.handle, arr, 64, ctypes.byref(cnt)))
        out = {}
        for k in range(min(cnt.value, 64)):
            out[arr[k].name.decode()] = {"launches": int(arr[k].launches), "ms": float(arr[k].ms),
                                         "bytes": float(arr[k].bytes)}
        return out

    def batch_run(self, circuits, dtype: int, flags: int = 0, params=None) -> np.ndarray:
        """Run a batch (a BatchSpec, or a sequence of circuit objects with n,
        gates, params, observable) in one persistent launch; returns
        out[b] = <O_b>.  `params` replaces the spec's concatenated angles."""
        spec = circuits if isinstance(circuits, BatchSpec) else BatchSpec(circuits)
        p = spec.params if params is None else np.ascontiguousarray(params, dtype=np.float64)
        out = np.zeros(spec.nb, dtype=np.float64)
        self.check(lib().qsv_batch_run(self.handle, spec.nb, _ptr(spec.nq), _ptr(spec.goff),
                                       _ptr(spec.gates), _ptr(p), p.size, _ptr(spec.toff),
                                       _ptr(spec.masks), _ptr(spec.w), dtype, _ptr(out), flags))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().qsv_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSpec:
    """Marshalled form of a batch of circuits for qsv_batch_run: qubit
    counts, gate records and offsets, concatenated angles (rotation indices
    rebased onto them), observable terms and offsets."""

    def __init__(self, circuits: Sequence):
        self.nb = len(circuits)
        self.nq = np.array([c.n for c in circuits], dtype=np.int32)
        gates, params, masks, ws = [], [], [], []
        goff, toff = [0], [0]
        pbase = 0
        for c in circuits:
            g = marshal_gates(c.gates)
            rot = g["kind"] == GROT
            g["param"][rot] += pbase
            p = np.asarray(c.params, dtype=np.float64)
            pbase += p.size
            gates.append(g)
            params.append(p)
            m, w = observable_arrays(c.observable)
            masks.append(m)
            ws.append(w)
            goff.append(goff[-1] + len(g))
            toff.append(toff[-1] + len(w))
        self.gates = np.concatenate(gates) if gates else np.zeros(0, dtype=GATE_DTYPE)
        self.params = np.concatenate(params) if params else np.zeros(0)
        self.masks = np.concatenate(masks).astype(np.uint64)
        self.w = np.concatenate(ws)
        self.goff = np.asarray(goff, dtype=np.int64)
        self.toff = np.asarray(toff, dtype=np.int64)


class State:
    """An n-qubit state in device memory (a torch tensor wrapped by qsv)."""

    def __init__(self, ctx: Context, n: int, dtype: int = QSV_C128, tensor=None):
        torch = _torch()
        self.ctx = ctx
        self.n = n
        self.dtype = dtype
        tdt = torch.complex128 if dtype == QSV_C128 else torch.complex64
        if tensor is None:
            tensor = torch.empty(2 ** n, dtype=tdt, device="cuda")
        if tensor.dtype != tdt or not tensor.is_contiguous() or tensor.numel() < 2 ** n:
            raise ValueError("state tensor must be contiguous, of the matching complex dtype, "
                             "with at least 2^n elements")
        self.tensor = tensor
        h = ctypes.c_void_p()
        ctx.check(lib().qsv_state_wrap(ctx.handle, ctypes.c_void_p(tensor.data_ptr()),
                                       tensor.numel() * tensor.element_size(), n, dtype,
                                       ctypes.byref(h)))
        self.handle = h

    # ---- gates
    def init_basis(self, b: int = 0):
        self.ctx.check(lib().qsv_init_basis(self.handle, b))

    def apply1q(self, q: int, u):
        self.ctx.check(lib().qsv_apply1q(self.handle, q, _ptr(_mat(u, 2))))

    def applyC1q(self, qc: int, qt: int, u, ctrl_state: int = 1):
        self.ctx.check(lib().qsv_applyC1q(self.handle, qc, qt, ctrl_state, _ptr(_mat(u, 2))))

    def apply2q(self, qa: int, qb: int, u):
        self.ctx.check(lib().qsv_apply2q(self.handle, qa, qb, _ptr(_mat(u, 4))))

    def applyMC1q(self, controls: Sequence[int], qt: int, u, ctrl_states: Optional[Sequence[int]] = None):
        c = np.ascontiguousarray(list(controls), dtype=np.int32)
        v = None if ctrl_states is None else np.ascontiguousarray(list(ctrl_states), dtype=np.int32)
        self.ctx.check(lib().qsv_applyMC1q(self.handle, c.size, _ptr(c), _ptr(v), qt, _ptr(_mat(u, 2))))

    def applyKq(self, qubits: Sequence[int], u):
        qs = np.ascontiguousarray(list(qubits), dtype=np.int32)
        self.ctx.check(lib().qsv_applyKq(self.handle, qs.size, _ptr(qs), _ptr(_mat(u, 2 ** qs.size))))

    def apply_circuit(self, gates, params=None, flags: int = 0, marshalled: Optional[np.ndarray] = None):
        g = marshalled if marshalled is not None else marshal_gates(gates)
        p = np.ascontiguousarray(np.zeros(0) if params is None else params, dtype=np.float64)
        self.ctx.check(lib().qsv_apply_circuit(self.handle, _ptr(g), len(g), _ptr(p), p.size, flags))

    # ---- reductions
    def norm2(self) -> float:
        out = ctypes.c_double()
        self.ctx.check(lib().qsv_norm2(self.handle, ctypes.byref(out)))
        return out.value

    def expect_z(self, obs) -> tuple:
        """obs: [(qubits, weight)] -> (per-term <Z...>, weighted sum)."""
        masks, w = observable_arrays(obs)
        terms = np.zeros(len(w))
        s = ctypes.c_double()
        self.ctx.check(lib().qsv_expect_z(self.handle, len(w), _ptr(masks), _ptr(w), _ptr(terms),
                                          ctypes.byref(s)))
        return terms, s.value

    def inner(self, other: "State") -> complex:
        out = np.zeros(2)
        self.ctx.check(lib().qsv_inner(self.handle, other.handle, _ptr(out)))
        return complex(out[0], out[1])

    def prob1(self, q: int) -> float:
        out = ctypes.c_double()
        self.ctx.check(lib().qsv_prob1(self.handle, q, ctypes.byref(out)))
        return out.value

    def measure1(self, q: int, r: float) -> int:
        out = ctypes.c_int()
        self.ctx.check(lib().qsv_measure1(self.handle, q, float(r), ctypes.byref(out)))
        return out.value

    def to_numpy(self) -> np.ndarray:
        npdt = np.complex128 if self.dtype == QSV_C128 else np.complex64
        out = np.empty(2 ** self.n, dtype=npdt)
        self.ctx.check(lib().qsv_copy_to_host(self.handle, _ptr(out), out.nbytes))
        return out

    def from_numpy(self, a: np.ndarray):
        npdt = np.complex128 if self.dtype == QSV_C128 else np.complex64
        a = np.ascontiguousarray(a, dtype=npdt)
        if a.size != 2 ** self.n:
            raise ValueError("wrong number of amplitudes")
        self.ctx.check(lib().qsv_copy_from_host(self.handle, _ptr(a), a.nbytes))

    def free(self):
        if getattr(self, "handle", None):
            lib().qsv_state_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def plan_circuit(n: int, gates, dtype: int = QSV_C128, tile_bits: int = 0, low_bits: int = 0,
                 reg_bits: int = 0):
    """Host-only pass plan of the gates as given, one to one (see
    qsv_plan_circuit): (pass_of_gate, exec_order, pass_qubit_masks)."""
    g = marshal_gates(gates)
    ng = len(g)
    pog = np.zeros(max(ng, 1), dtype=np.int32)
    order = np.zeros(max(ng, 1), dtype=np.int32)
    pq = np.zeros(max(ng, 1), dtype=np.uint64)
    npass = ctypes.c_int64()
    st = lib().qsv_plan_circuit(n, dtype, _ptr(g), ng, tile_bits, low_bits, reg_bits, ctypes.byref(npass),
                                _ptr(pog), _ptr(order), _ptr(pq))
    if st != QSV_OK:
        raise QsvError(st, "qsv_plan_circuit failed")
    return pog[:ng], order[:ng], pq[: npass.value]


def plan_fused(n: int, gates, params=None, dtype: int = QSV_C128, tile_bits: int = 0,
               low_bits: int = 0, reg_bits: int = 0, lds_rounds: int = 0):
    """Host-only: the exact gate records the kernels apply, in order, and the
    pass index of each (see qsv_plan_fused)."""
    g = marshal_gates(gates)
    p = np.ascontiguousarray(np.zeros(0) if params is None else params, dtype=np.float64)
    cap = 2 * len(g) + 8
    nout = ctypes.c_int64()
    for _ in range(2):   # a second try with the count the first one reported
        out = np.zeros(cap, dtype=GATE_DTYPE)
        pas = np.zeros(cap, dtype=np.int32)
        st = lib().qsv_plan_fused(n, dtype, _ptr(g), len(g), _ptr(p), p.size, tile_bits, low_bits,
                                  reg_bits, lds_rounds, _ptr(out), cap, _ptr(pas), ctypes.byref(nout))
        if st == QSV_OK or nout.value <= cap:
            break
        cap = int(nout.value)
    if st != QSV_OK:
        raise QsvError(st, "qsv_plan_fused failed")
    return out[: nout.value], pas[: nout.value]


def jit_source(n: int, gates, pass_index: int, dtype: int = QSV_C128, params=None) -> str:
    """Generated source of fused pass `pass_index` (host only)."""
    g = marshal_gates(gates)
    p = np.ascontiguousarray(np.zeros(0) if params is None else params, dtype=np.float64)
    ln = ctypes.c_size_t()
    st = lib().qsv_jit_source(n, dtype, _ptr(g), len(g), _ptr(p), p.size, pass_index, None, 0,
                              ctypes.byref(ln))
    if st != QSV_OK:
        raise QsvError(st, "qsv_jit_source failed")
    buf = ctypes.create_string_buffer(ln.value + 1)
    st = lib().qsv_jit_source(n, dtype, _ptr(g), len(g), _ptr(p), p.size, pass_index, buf,
                              ln.value + 1, ctypes.byref(ln))
    if st != QSV_OK:
        raise QsvError(st, "qsv_jit_source failed")
    return buf.value.decode()


def adjoint(psi: State, lam: State, gates, params, obs, flags: int = FLAG_FORWARD,
            marshalled: Optional[np.ndarray] = None):
    """(f, grad) by the adjoint sweep; see qsv_adjoint."""
    g = marshalled if marshalled is not None else marshal_gates(gates)
    p = np.ascontiguousarray(np.zeros(0) if params is None else params, dtype=np.float64)
    masks, w = observable_arrays(obs)
    grad = np.zeros(max(p.size, 1))
    f = ctypes.c_double()
    psi.ctx.check(lib().qsv_adjoint(psi.handle, lam.handle, _ptr(g), len(g), _ptr(p), p.size,
                                    len(w), _ptr(masks), _ptr(w), ctypes.byref(f), _ptr(grad),
                                    flags))
    return f.value, grad[: p.size]
