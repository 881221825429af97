"""Index maps of the paper's gate algorithms, as plain enumerations.

These are the zero-bit-insertion index sets of Algs. 1-3 (Sec. 2.1-2.3),
written out with Python integers so they can be checked against the worked
examples printed in Figs. 3-5 and against the partition property (the pair or
quad sets of one gate cover every index exactly once, which is also what
makes an in-place update race-free).  Test infrastructure only.
"""
from __future__ import annotations

from typing import List, Tuple


def masks_1q(n: int, q: int) -> Tuple[int, int]:
    """(m_L, m_R) of Sec. 2.1: m_R keeps the n-q-1 bits right of qubit q,
    m_L the q bits left of it (in the (n-1)-bit loop counter j)."""
    m_r = 2 ** (n - q - 1) - 1
    m_l = (2 ** (n - 1) - 1) - m_r
    return m_l, m_r


def pairs_1q(n: int, q: int) -> List[Tuple[int, int]]:
    """[(a_j, b_j)] for j = 0..2^(n-1)-1 (Alg. 1)."""
    m_l, m_r = masks_1q(n, q)
    out = []
    for j in range(2 ** (n - 1)):
        a = (j & m_r) + ((j & m_l) << 1)
        out.append((a, a + 2 ** (n - q - 1)))
    return out


def masks_2(n: int, qa: int, qb: int) -> Tuple[int, int, int]:
    """(m_L, m_C, m_R) of Sec. 2.2 for the ordered pair q0 = min < q1 = max."""
    q0, q1 = min(qa, qb), max(qa, qb)
    m_r = 2 ** (n - q1 - 1) - 1
    m_c = (2 ** (n - q0 - 2) - 1) - m_r
    m_l = (2 ** (n - 2) - 1) - m_r - m_c
    return m_l, m_c, m_r


def _base(j: int, m_l: int, m_c: int, m_r: int) -> int:
    return (j & m_r) + ((j & m_c) << 1) + ((j & m_l) << 2)


def pairs_c1q(n: int, qc: int, qt: int, cs: int) -> List[Tuple[int, int]]:
    """[(a_j, b_j)] for j = 0..2^(n-2)-1 (Alg. 2): zero bits inserted at both
    qubits, b_j adds the target weight, and control state 1 adds the control
    weight to both."""
    m_l, m_c, m_r = masks_2(n, qc, qt)
    out = []
    for j in range(2 ** (n - 2)):
        a = _base(j, m_l, m_c, m_r)
        b = a + 2 ** (n - qt - 1)
        if cs == 1:
            a += 2 ** (n - qc - 1)
            b += 2 ** (n - qc - 1)
        out.append((a, b))
    return out


def quads_2q_as_printed(n: int, q0: int, q1: int) -> List[Tuple[int, int, int, int]]:
    """[(a_j, b_j, c_j, d_j)] exactly as Alg. 3 prints them for q0 < q1:
    b_j sets q0's bit, c_j sets q1's bit."""
    m_l, m_c, m_r = masks_2(n, q0, q1)
    out = []
    for j in range(2 ** (n - 2)):
        a = _base(j, m_l, m_c, m_r)
        w0, w1 = 2 ** (n - q0 - 1), 2 ** (n - q1 - 1)
        out.append((a, a + w0, a + w1, a + w0 + w1))
    return out


def quads_2q(n: int, qa: int, qb: int) -> List[Tuple[int, int, int, int]]:
    """Quads in the local order 2*x_qa + x_qb (the reading eq. (1) fixes for a
    2-qubit gate on (qa, qb)): entry r of a quad is the index whose qa bit is
    r >> 1 and whose qb bit is r & 1."""
    m_l, m_c, m_r = masks_2(n, qa, qb)
    wa, wb = 2 ** (n - qa - 1), 2 ** (n - qb - 1)
    out = []
    for j in range(2 ** (n - 2)):
        a = _base(j, m_l, m_c, m_r)
        out.append((a, a + wb, a + wa, a + wa + wb))
    return out
