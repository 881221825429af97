"""OpenQASM 2.0 front-end: program text -> qsv_gate records for
qsv_apply_circuit.

The engine applies 1-qubit, controlled 1-qubit and 2-qubit gates on any
qubits (Sec. 2.1-2.3) and gates with extra controls (Sec. 2.4); this module
lowers an OpenQASM 2.0 program onto exactly those records.  It is host-side
parsing only: every gate still runs in the HIP kernels.

Supported
  - `OPENQASM 2.0;`, `include "...";` (the standard gate names below are
    built in, so the include is not read), `qreg`, `creg`, `barrier`
    (ignored), `measure` (recorded in `Program.measures`, not applied: the
    state vector keeps every amplitude), user `gate` definitions (expanded
    like macros, with parameters and nested calls), register broadcasting
    (`h q;`, `cx a, b;` over equal-size registers).
  - Parameter expressions: numbers, `pi`, + - * / ^, unary minus,
    parentheses and sin, cos, tan, exp, ln, sqrt.
  - Built-in gates, with c, s = cos(t/2), sin(t/2):
      U, u3, u (t, p, l) = [[c, -e^{il} s], [e^{ip} s, e^{i(p+l)} c]]
      u2(p, l) = u3(pi/2, p, l);  u1, p(l) = diag(1, e^{il});  id, u0 = I
      x, y, z, h, s, sdg, t, tdg, sx, sxdg (textbook matrices)
      rx, ry, rz (t) = exp(-i t P / 2)
      CX, cx, cy, cz, ch, csx, crx, cry, crz, cu1, cp, cu3, cu(t, p, l, g)
        -> controlled 1-qubit gates (cu: e^{ig} u3 on the target)
      swap, rxx(t) = exp(-i t XX/2), rzz(t) = exp(-i t ZZ/2), iswap
        -> 2-qubit gates
      ccx, c3x, c4x (X with 2, 3, 4 controls), cswap (SWAP with a control),
      c3sqrtx (sx with 3 controls) -> gates with extra controls
    Gates that differ from a textbook one only by a global phase (rz and u1,
    for instance) are applied as written above; controlled forms keep their
    relative phases.
Not supported (an error names the statement): `opaque`, `reset`, `if`.
"""
from __future__ import annotations

import math
import re
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .qsv import G1Q, G2Q, GATE_DTYPE, GC1Q


class QasmError(ValueError):
    pass


@dataclass
class Program:
    n: int                                   # total qubits (registers in declaration order)
    gates: np.ndarray                        # qsv_gate records (GATE_DTYPE)
    qregs: Dict[str, Tuple[int, int]]        # name -> (first qubit, size)
    cregs: Dict[str, int]                    # name -> size
    measures: List[Tuple[int, Tuple[str, int]]] = field(default_factory=list)


# ------------------------------------------------------------ gate matrices
_SQ2 = 1.0 / math.sqrt(2.0)
_I2 = np.eye(2, dtype=complex)
_X = np.array([[0, 1], [1, 0]], dtype=complex)
_Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
_Z = np.array([[1, 0], [0, -1]], dtype=complex)
_H = np.array([[1, 1], [1, -1]], dtype=complex) * _SQ2
_SX = np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=complex) / 2.0
_SWAP = np.eye(4, dtype=complex)[[0, 2, 1, 3]]


def _u3(t, p, l):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -np.exp(1j * l) * s], [np.exp(1j * p) * s, np.exp(1j * (p + l)) * c]])


def _phase(l):
    return np.diag([1.0, np.exp(1j * l)])


def _rot(P, t):
    return math.cos(t / 2) * np.eye(P.shape[0]) - 1j * math.sin(t / 2) * P


# name -> (number of parameters, number of qubits, builder)
# builder(params) -> ("1q", U) | ("c1q", U) | ("2q", U4) | ("mc", U, ncontrols) | ("mc2q", U4, nc)
_BUILTIN = {
    "U": (3, 1, lambda a: ("1q", _u3(*a))),
    "u3": (3, 1, lambda a: ("1q", _u3(*a))),
    "u": (3, 1, lambda a: ("1q", _u3(*a))),
    "u2": (2, 1, lambda a: ("1q", _u3(math.pi / 2, a[0], a[1]))),
    "u1": (1, 1, lambda a: ("1q", _phase(a[0]))),
    "p": (1, 1, lambda a: ("1q", _phase(a[0]))),
    "id": (0, 1, lambda a: ("1q", _I2)),
    "u0": (1, 1, lambda a: ("1q", _I2)),
    "x": (0, 1, lambda a: ("1q", _X)),
    "y": (0, 1, lambda a: ("1q", _Y)),
    "z": (0, 1, lambda a: ("1q", _Z)),
    "h": (0, 1, lambda a: ("1q", _H)),
    "s": (0, 1, lambda a: ("1q", _phase(math.pi / 2))),
    "sdg": (0, 1, lambda a: ("1q", _phase(-math.pi / 2))),
    "t": (0, 1, lambda a: ("1q", _phase(math.pi / 4))),
    "tdg": (0, 1, lambda a: ("1q", _phase(-math.pi / 4))),
    "sx": (0, 1, lambda a: ("1q", _SX)),
    "sxdg": (0, 1, lambda a: ("1q", _SX.conj().T)),
    "rx": (1, 1, lambda a: ("1q", _rot(_X, a[0]))),
    "ry": (1, 1, lambda a: ("1q", _rot(_Y, a[0]))),
    "rz": (1, 1, lambda a: ("1q", _rot(_Z, a[0]))),
    "CX": (0, 2, lambda a: ("c1q", _X)),
    "cx": (0, 2, lambda a: ("c1q", _X)),
    "cy": (0, 2, lambda a: ("c1q", _Y)),
    "cz": (0, 2, lambda a: ("c1q", _Z)),
    "ch": (0, 2, lambda a: ("c1q", _H)),
    "csx": (0, 2, lambda a: ("c1q", _SX)),
    "crx": (1, 2, lambda a: ("c1q", _rot(_X, a[0]))),
    "cry": (1, 2, lambda a: ("c1q", _rot(_Y, a[0]))),
    "crz": (1, 2, lambda a: ("c1q", _rot(_Z, a[0]))),
    "cu1": (1, 2, lambda a: ("c1q", _phase(a[0]))),
    "cp": (1, 2, lambda a: ("c1q", _phase(a[0]))),
    "cu3": (3, 2, lambda a: ("c1q", _u3(*a))),
    "cu": (4, 2, lambda a: ("c1q", np.exp(1j * a[3]) * _u3(a[0], a[1], a[2]))),
    "swap": (0, 2, lambda a: ("2q", _SWAP)),
    "iswap": (0, 2, lambda a: ("2q", np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]]))),
    "rxx": (1, 2, lambda a: ("2q", _rot(np.kron(_X, _X), a[0]))),
    "rzz": (1, 2, lambda a: ("2q", _rot(np.kron(_Z, _Z), a[0]))),
    "ccx": (0, 3, lambda a: ("mc", _X, 2)),
    "c3x": (0, 4, lambda a: ("mc", _X, 3)),
    "c4x": (0, 5, lambda a: ("mc", _X, 4)),
    "c3sqrtx": (0, 4, lambda a: ("mc", _SX, 3)),
    "cswap": (0, 3, lambda a: ("mc2q", _SWAP, 1)),
}


# ------------------------------------------------------- expressions
_TOKEN = re.compile(r"\s*(?:(\d+\.\d*(?:[eE][-+]?\d+)?|\.\d+(?:[eE][-+]?\d+)?|\d+(?:[eE][-+]?\d+)?)"
                    r"|([A-Za-z_][A-Za-z0-9_]*)|(\S))")
_FUNCS = {"sin": math.sin, "cos": math.cos, "tan": math.tan, "exp": math.exp, "ln": math.log,
          "sqrt": math.sqrt}


def eval_expr(text: str, env: Dict[str, float]) -> float:
    """Evaluate an OpenQASM 2.0 parameter expression (recursive descent)."""
    toks = []
    pos = 0
    text = text.strip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            raise QasmError(f"bad expression {text!r}")
        num, name, op = m.groups()
        toks.append(("n", float(num)) if num else ("id", name) if name else ("op", op))
        pos = m.end()
    toks.append(("end", None))
    i = 0

    def peek():
        return toks[i]

    def take():
        nonlocal i
        t = toks[i]
        i += 1
        return t

    def expect(op):
        t = take()
        if t != ("op", op):
            raise QasmError(f"expected {op!r} in {text!r}")

    def atom():
        t = take()
        if t[0] == "n":
            return t[1]
        if t == ("op", "("):
            v = add()
            expect(")")
            return v
        if t == ("op", "-"):
            return -power()
        if t == ("op", "+"):
            return power()
        if t[0] == "id":
            if t[1] == "pi":
                return math.pi
            if t[1] in _FUNCS:
                expect("(")
                v = add()
                expect(")")
                return _FUNCS[t[1]](v)
            if t[1] in env:
                return env[t[1]]
            raise QasmError(f"unknown name {t[1]!r} in {text!r}")
        raise QasmError(f"bad expression {text!r}")

    def power():
        b = atom()
        if peek() == ("op", "^"):
            take()
            return b ** power()
        return b

    def mul():
        v = power()
        while peek() in (("op", "*"), ("op", "/")):
            op = take()[1]
            r = power()
            v = v * r if op == "*" else v / r
        return v

    def add():
        v = mul()
        while peek() in (("op", "+"), ("op", "-")):
            op = take()[1]
            r = mul()
            v = v + r if op == "+" else v - r
        return v

    v = add()
    if peek()[0] != "end":
        raise QasmError(f"trailing text in expression {text!r}")
    return float(v)


def _split_args(s: str) -> List[str]:
    """Split on top-level commas."""
    out, depth, cur = [], 0, []
    for ch in s:
        if ch == "(":
            depth += 1
        elif ch == ")":
            depth -= 1
        if ch == "," and depth == 0:
            out.append("".join(cur).strip())
            cur = []
        else:
            cur.append(ch)
    if "".join(cur).strip():
        out.append("".join(cur).strip())
    return out


# ------------------------------------------------------------- the parser
_STMT_GATE = re.compile(r"^([A-Za-z_][A-Za-z0-9_]*)\s*(?:\((.*)\))?\s+(.+)$", re.S)


@dataclass
class _GateDef:
    params: List[str]
    qargs: List[str]
    body: List[str]


def _strip_comments(text: str) -> str:
    return re.sub(r"//[^\n]*", "", text)


def _statements(text: str) -> List[str]:
    """Top-level statements; a gate definition is one statement including
    its braced body."""
    out, cur, depth = [], [], 0
    for ch in text:
        cur.append(ch)
        if ch == "{":
            depth += 1
        elif ch == "}":
            depth -= 1
            if depth == 0:
                out.append("".join(cur).strip())
                cur = []
        elif ch == ";" and depth == 0:
            out.append("".join(cur)[:-1].strip())
            cur = []
    if "".join(cur).strip():
        raise QasmError(f"unterminated statement: {''.join(cur).strip()[:60]!r}")
    return [s for s in out if s]


def parse(text: str) -> Program:
    """Parse an OpenQASM 2.0 program into qsv_gate records."""
    text = _strip_comments(text)
    qregs: Dict[str, Tuple[int, int]] = {}
    cregs: Dict[str, int] = {}
    defs: Dict[str, _GateDef] = {}
    recs: List[tuple] = []   # (kind, qubits, matrix, controls)
    measures = []
    nq = 0

    def operand(tok: str) -> List[int]:
        m = re.fullmatch(r"\s*([A-Za-z_][A-Za-z0-9_]*)\s*(?:\[\s*(\d+)\s*\])?\s*", tok)
        if not m or m.group(1) not in qregs:
            raise QasmError(f"unknown qubit operand {tok!r}")
        base, size = qregs[m.group(1)]
        if m.group(2) is None:
            return [base + i for i in range(size)]
        i = int(m.group(2))
        if i >= size:
            raise QasmError(f"index out of range in {tok!r}")
        return [base + i]

    def emit(name: str, args: List[float], qs: List[int], depth: int):
        if depth > 64:
            raise QasmError("gate definitions nest too deeply")
        if len(set(qs)) != len(qs):
            raise QasmError(f"repeated qubit in {name} {qs}")
        if name in defs:
            d = defs[name]
            if len(args) != len(d.params) or len(qs) != len(d.qargs):
                raise QasmError(f"{name}: wrong number of parameters or qubits")
            env = dict(zip(d.params, args))
            qmap = dict(zip(d.qargs, qs))
            for st in d.body:
                call(st, env, qmap, depth + 1)
            return
        if name not in _BUILTIN:
            raise QasmError(f"unknown gate {name!r}")
        npar, nqb, build = _BUILTIN[name]
        if len(args) != npar or len(qs) != nqb:
            raise QasmError(f"{name}: expects {npar} parameters and {nqb} qubits")
        spec = build(args)
        kind = spec[0]
        if kind == "1q":
            recs.append((G1Q, (qs[0],), spec[1], ()))
        elif kind == "c1q":
            recs.append((GC1Q, (qs[0], qs[1]), spec[1], ()))
        elif kind == "2q":
            recs.append((G2Q, (qs[0], qs[1]), spec[1], ()))
        elif kind == "mc":
            nc = spec[2]
            recs.append((G1Q, (qs[nc],), spec[1], tuple(qs[:nc])))
        else:   # mc2q
            nc = spec[2]
            recs.append((G2Q, (qs[nc], qs[nc + 1]), spec[1], tuple(qs[:nc])))

    def call(stmt: str, env: Dict[str, float], qmap, depth: int):
        stmt = stmt.strip()
        if not stmt:
            return
        if stmt.startswith("barrier"):
            return
        m = _STMT_GATE.match(stmt)
        if not m:
            raise QasmError(f"cannot parse {stmt!r}")
        name, ptxt, qtxt = m.group(1), m.group(2), m.group(3)
        args = [eval_expr(a, env) for a in _split_args(ptxt)] if ptxt and ptxt.strip() else []
        ops = _split_args(qtxt)
        if qmap is not None:   # inside a gate body: formal qubit names
            try:
                qs = [qmap[o.strip()] for o in ops]
            except KeyError as e:
                raise QasmError(f"unknown qubit {e} in gate body") from None
            emit(name, args, qs, depth)
            return
        lists = [operand(o) for o in ops]
        width = max(len(x) for x in lists)
        if any(len(x) not in (1, width) for x in lists):
            raise QasmError(f"register sizes differ in {stmt!r}")
        for i in range(width):
            emit(name, args, [x[0] if len(x) == 1 else x[i] for x in lists], depth)

    for stmt in _statements(text):
        head = stmt.split(None, 1)[0] if stmt.split() else ""
        if head == "OPENQASM":
            if not stmt.split()[1].startswith("2"):
                raise QasmError("only OpenQASM 2.x is supported")
        elif head == "include":
            continue
        elif head in ("qreg", "creg"):
            m = re.fullmatch(r"(qreg|creg)\s+([A-Za-z_][A-Za-z0-9_]*)\s*\[\s*(\d+)\s*\]", stmt)
            if not m:
                raise QasmError(f"bad register declaration {stmt!r}")
            if m.group(2) in qregs or m.group(2) in cregs:
                raise QasmError(f"register {m.group(2)!r} declared twice")
            if m.group(1) == "qreg":
                qregs[m.group(2)] = (nq, int(m.group(3)))
                nq += int(m.group(3))
            else:
                cregs[m.group(2)] = int(m.group(3))
        elif head == "gate":
            m = re.fullmatch(r"gate\s+([A-Za-z_][A-Za-z0-9_]*)\s*(?:\(([^)]*)\))?\s*([^{]*)\{(.*)\}", stmt, re.S)
            if not m:
                raise QasmError(f"bad gate definition {stmt[:60]!r}")
            params = [p.strip() for p in m.group(2).split(",")] if m.group(2) and m.group(2).strip() else []
            qargs = [a.strip() for a in m.group(3).split(",") if a.strip()]
            body = [b for b in m.group(4).split(";") if b.strip()]
            defs[m.group(1)] = _GateDef(params, qargs, body)
        elif head == "measure":
            m = re.fullmatch(r"measure\s+(.+?)\s*->\s*(.+)", stmt)
            if not m:
                raise QasmError(f"bad measure {stmt!r}")
            qs = operand(m.group(1))
            cm = re.fullmatch(r"\s*([A-Za-z_][A-Za-z0-9_]*)\s*(?:\[\s*(\d+)\s*\])?\s*", m.group(2))
            if not cm or cm.group(1) not in cregs:
                raise QasmError(f"unknown classical operand in {stmt!r}")
            for i, qb in enumerate(qs):
                measures.append((qb, (cm.group(1), int(cm.group(2)) if cm.group(2) else i)))
        elif head in ("opaque", "reset", "if"):
            raise QasmError(f"unsupported statement {head!r}")
        else:
            call(stmt, {}, None, 0)

    g = np.zeros(len(recs), dtype=GATE_DTYPE)
    for i, (kind, qs, u, ctrls) in enumerate(recs):
        g["kind"][i] = kind
        g["q0"][i] = qs[0]
        if len(qs) > 1:
            g["q1"][i] = qs[1]
        g["ctrl_state"][i] = 1
        g["param"][i] = -1
        u = np.asarray(u, dtype=complex)
        g["m"][i][: 2 * u.size] = np.stack([u.real, u.imag], axis=-1).reshape(-1)
        for c in ctrls:
            g["cmask"][i] |= np.uint64(1 << c)
            g["cvals"][i] |= np.uint64(1 << c)
    return Program(nq, g, qregs, cregs, measures)


def load(path: str) -> Program:
    with open(path) as f:
        return parse(f.read())
