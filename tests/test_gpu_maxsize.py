"""The largest states the interface accepts that fit one MI355X (288 GB of
HBM): 34 qubits in complex128 and 35 in complex64, 256 GiB each.  No CPU
oracle holds such a state, so the checks use amplitudes the oracle computes
one by one:

  * one layer of Haar 1-qubit gates on every qubit (fused tile passes), then
    a Haar 2-qubit gate and a controlled gate on the extreme qubits 0 and
    n-1 (one kernel per gate, index bits n-1 and 0).  Each sampled amplitude
    then depends on four product amplitudes, which the oracle combines with
    its own gate applications on the 2-qubit subsystem of qubits 0 and n-1;
  * the norm stays 1;
  * P(qubit 0 = 1) equals the marginal of that subsystem, and a measurement
    of qubit 0 zeroes the other branch and rescales the kept one.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

GIB = 2 ** 30


def _device_or_skip(state_bytes: int):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < state_bytes + 4 * GIB:
        pytest.skip(f"needs {state_bytes / GIB + 4:.0f} GiB of free device memory, "
                    f"{free / GIB:.0f} GiB free")


@pytest.mark.parametrize("dt_name,n,tol_amp,tol_norm",
                         [("c128", 34, 1e-12, 1e-11), ("c64", 35, 1e-9, 1e-5)])
def test_largest_state_sampled_amplitudes(dt_name, n, tol_amp, tol_norm):
    import torch
    import paper_2303_00123_amd as q
    dt = q.QSV_C128 if dt_name == "c128" else q.QSV_C64
    _device_or_skip((2 ** n) * (16 if dt == q.QSV_C128 else 8))
    rng = np.random.default_rng(3400 + n)
    us = [W.haar_unitary(2, rng) for _ in range(n)]
    u2 = W.haar_unitary(4, rng)
    v = W.haar_unitary(2, rng)
    qstates = np.array([O.apply_1q(O.basis(1), 0, u) for u in us])

    ctx = q.Context()
    st = q.State(ctx, n, dt)
    try:
        st.init_basis(0)
        st.apply_circuit([W.g1(qb, us[qb]) for qb in range(n)])
        st.apply2q(0, n - 1, u2)
        st.applyC1q(n - 1, 0, v, ctrl_state=1)
        xs = np.concatenate([[0, 2 ** n - 1, 1, 2 ** (n - 1)],
                             rng.integers(0, 2 ** n, size=40)]).astype(np.int64)
        got = st.tensor[torch.as_tensor(xs, device="cuda")].cpu().numpy().astype(np.complex128)
        hi, lo = 1 << (n - 1), 1          # index bits of qubit 0 and qubit n-1
        ref = []
        for x in map(int, xs):
            base = x & ~(hi | lo)
            sub = np.array([O.product_amplitude(qstates, base | (hi if a else 0) | (lo if b else 0))
                            for a in (0, 1) for b in (0, 1)])
            # subsystem qubit 0 = qubit 0, subsystem qubit 1 = qubit n-1
            sub = O.apply_2q(sub, 0, 1, u2)
            sub = O.apply_c1q(sub, 1, 0, v, 1)
            ref.append(sub[2 * ((x >> (n - 1)) & 1) + (x & 1)])
        ref = np.array(ref)
        assert np.max(np.abs(got - ref)) < tol_amp
        assert abs(st.norm2() - 1.0) < tol_norm
        # the marginal of qubits (0, n-1): the other qubits stay a product of
        # unit vectors, so P(qubit 0 = 1) comes from the 2-qubit subsystem
        sub = np.kron(qstates[0], qstates[n - 1])
        sub = O.apply_c1q(O.apply_2q(sub, 0, 1, u2), 1, 0, v, 1)
        p1 = float(abs(sub[2]) ** 2 + abs(sub[3]) ** 2)
        assert abs(st.prob1(0) - p1) < (1e-12 if dt == q.QSV_C128 else 1e-5)
        # measurement: outcome by r against P(0), then collapse and renormalise
        r = 0.5 * (1.0 - p1) if p1 < 0.5 else 0.5 * (1.0 - p1) + p1   # far from the boundary
        outcome = st.measure1(0, r)
        assert outcome == (0 if r < 1.0 - p1 else 1)
        assert abs(st.norm2() - 1.0) < tol_norm
        got = st.tensor[torch.as_tensor(xs, device="cuda")].cpu().numpy().astype(np.complex128)
        bit = (xs >> (n - 1)) & 1
        keep = np.sqrt(p1 if outcome else 1.0 - p1)
        assert np.max(np.abs(got[bit != outcome])) == 0.0
        assert np.max(np.abs(got[bit == outcome] - ref[bit == outcome] / keep)) < 10 * tol_amp
    finally:
        st.free()
        ctx.close()
        del st
        torch.cuda.empty_cache()


@pytest.mark.parametrize("dt_name,tol", [("c128", 1e-12), ("c64", 2e-6)])
def test_adjoint_32_qubits_closed_form(dt_name, tol):
    """Adjoint sweep at 32 qubits (two 64 GiB / 32 GiB vectors), fused and one
    kernel per gate.  RY rotations on qubits 0, 1, 30 and 31 (and an RZ on
    qubit 1) from |0...0> leave a product state, so with
    O = 0.8 Z0 Z31 - 0.5 Z1 + 0.3 Z30 the value is
    0.8 cos a cos d - 0.5 cos b + 0.3 cos c and the gradient is closed-form
    (RY(t)|0> has <Z> = cos t; the RZ angle has gradient 0)."""
    import torch
    import paper_2303_00123_amd as q
    n = 32
    dt = q.QSV_C128 if dt_name == "c128" else q.QSV_C64
    _device_or_skip(2 * (2 ** n) * (16 if dt == q.QSV_C128 else 8))
    gates = [W.grot(0, "Y", 0), W.grot(1, "Y", 1), W.grot(1, "Z", 2), W.grot(30, "Y", 3),
             W.grot(31, "Y", 4)]
    th = np.array([0.3, 1.1, 0.7, -0.4, 2.0])
    obs = [((0, 31), 0.8), ((1,), -0.5), ((30,), 0.3)]
    a, b, _, c, d = th
    f_ref = 0.8 * np.cos(a) * np.cos(d) - 0.5 * np.cos(b) + 0.3 * np.cos(c)
    g_ref = np.array([-0.8 * np.sin(a) * np.cos(d), 0.5 * np.sin(b), 0.0, -0.3 * np.sin(c),
                      -0.8 * np.cos(a) * np.sin(d)])
    ctx = q.Context()
    psi, lam = q.State(ctx, n, dt), q.State(ctx, n, dt)
    try:
        for flags in (q.FLAG_FORWARD, q.FLAG_FORWARD | q.FLAG_NO_FUSE):
            f, g = q.adjoint(psi, lam, gates, th, obs, flags=flags)
            assert abs(f - f_ref) < tol
            assert np.max(np.abs(g - g_ref)) < tol
    finally:
        psi.free()
        lam.free()
        ctx.close()
        del psi, lam
        torch.cuda.empty_cache()


@pytest.mark.parametrize("dt_name,n,tol_amp", [("c128", 33, 1e-12), ("c64", 34, 1e-9)])
def test_unfused_grid_stride_loops_sampled(dt_name, n, tol_amp):
    """One kernel per gate at 33 (c128) / 34 (c64) qubits, 128 GiB: the pair
    and quad counts exceed the capped grid, so every gate kernel loops over
    blocks.  A dense Haar gate on every qubit (Alg. 1), then a controlled
    gate with its control at index bit n-2 (Alg. 2, half the state moves) on
    qubits (1, n-2) and a 2-qubit gate (Alg. 3) on (2, n-3).  The two
    entangled pairs are disjoint, so each sampled amplitude is the oracle's
    product over the untouched qubits times the oracle's 2-qubit subsystem
    amplitudes of the two pairs."""
    import torch
    import paper_2303_00123_amd as q
    dt = q.QSV_C128 if dt_name == "c128" else q.QSV_C64
    _device_or_skip((2 ** n) * (16 if dt == q.QSV_C128 else 8))
    rng = np.random.default_rng(3300 + n)
    us = [W.haar_unitary(2, rng) for _ in range(n)]
    v = W.haar_unitary(2, rng)
    u2 = W.haar_unitary(4, rng)
    qstates = np.array([O.apply_1q(O.basis(1), 0, u) for u in us])
    # subsystems (qubit order within each pair as in the gates)
    s1 = O.apply_c1q(np.kron(qstates[1], qstates[n - 2]), 0, 1, v, 1)
    s2 = O.apply_2q(np.kron(qstates[2], qstates[n - 3]), 0, 1, u2)
    ones = np.array([1.0 + 0j, 1.0 + 0j])
    rest = qstates.copy()
    for qb in (1, n - 2, 2, n - 3):
        rest[qb] = ones
    ctx = q.Context()
    st = q.State(ctx, n, dt)
    try:
        st.init_basis(0)
        st.apply_circuit([W.g1(qb, us[qb]) for qb in range(n)], flags=q.FLAG_NO_FUSE)
        st.applyC1q(1, n - 2, v, ctrl_state=1)
        st.apply2q(2, n - 3, u2)
        xs = np.concatenate([[0, 2 ** n - 1, 1, 2 ** (n - 1), 2 ** (n - 2) + 2],
                             rng.integers(0, 2 ** n, size=40)]).astype(np.int64)
        got = st.tensor[torch.as_tensor(xs, device="cuda")].cpu().numpy().astype(np.complex128)
        bit = lambda x, qb: (x >> (n - 1 - qb)) & 1   # noqa: E731
        ref = np.array([O.product_amplitude(rest, int(x)) * s1[2 * bit(x, 1) + bit(x, n - 2)]
                        * s2[2 * bit(x, 2) + bit(x, n - 3)] for x in map(int, xs)])
        assert np.max(np.abs(got - ref)) < tol_amp
    finally:
        st.free()
        ctx.close()
        del st
        torch.cuda.empty_cache()


@pytest.mark.parametrize("dt_name,n,tol_amp", [("c128", 32, 1e-12), ("c64", 33, 1e-6)])
def test_matrix_core_kq_grid_stride_sampled(dt_name, n, tol_amp):
    """A dense 3-qubit gate on the matrix cores at 32 (c128) / 33 (c64)
    qubits, 64 GiB: 2^(n-3)/64 blocks exceed the capped grid, so the kernel
    walks several blocks per workgroup in XCD order.  A Haar gate on every
    qubit first (a product state), then U on qubits (n-1, 0, n//2) (lowest,
    highest and a middle index bit).  Each sampled amplitude is the oracle's
    product over the other qubits times the oracle's 3-qubit subsystem
    amplitude."""
    import torch
    import paper_2303_00123_amd as q
    dt = q.QSV_C128 if dt_name == "c128" else q.QSV_C64
    _device_or_skip((2 ** n) * (16 if dt == q.QSV_C128 else 8))
    rng = np.random.default_rng(3500 + n)
    us = [W.haar_unitary(2, rng) for _ in range(n)]
    u = W.haar_unitary(8, rng)
    qs = [n - 1, 0, n // 2]
    qstates = np.array([O.apply_1q(O.basis(1), 0, v) for v in us])
    sub = O.apply_kq(np.kron(np.kron(qstates[qs[0]], qstates[qs[1]]), qstates[qs[2]]), [0, 1, 2], u)
    ones = np.array([1.0 + 0j, 1.0 + 0j])
    rest = qstates.copy()
    for qb in qs:
        rest[qb] = ones
    ctx = q.Context()
    ctx.set_matrix_cores(1)
    st = q.State(ctx, n, dt)
    try:
        st.init_basis(0)
        st.apply_circuit([W.g1(qb, us[qb]) for qb in range(n)])
        ctx.profile_begin()
        st.applyKq(qs, u)
        assert list(ctx.profile_end()) == [f"kq_mfma_{dt_name}"]
        xs = np.concatenate([[0, 2 ** n - 1, 1, 2 ** (n - 1), 2 ** (n // 2)],
                             rng.integers(0, 2 ** n, size=60)]).astype(np.int64)
        got = st.tensor[torch.as_tensor(xs, device="cuda")].cpu().numpy().astype(np.complex128)
        bit = lambda x, qb: (x >> (n - 1 - qb)) & 1   # noqa: E731
        ref = np.array([O.product_amplitude(rest, int(x))
                        * sub[4 * bit(x, qs[0]) + 2 * bit(x, qs[1]) + bit(x, qs[2])] for x in map(int, xs)])
        assert np.max(np.abs(got - ref)) < tol_amp
    finally:
        st.free()
        ctx.close()
        del st
        torch.cuda.empty_cache()
