"""Specialised tile-pass kernels (qsv_set_jit): the generated kernel of each
fused pass against the FP64 oracle, in both precisions, over every tile
shape and both LDS exchanges; a circuit with the same structure and new
angles reuses the kernels; the result equals the interpreting kernel's."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL128 = 1e-12


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2303_00123_amd as qq
    return qq


def infidelity(a64, b128):
    ov = np.vdot(a64.astype(np.complex128), b128)
    return 1.0 - abs(ov) ** 2


def run(q, ctx, c, dtype, phi=None, flags=0, params=None):
    st = q.State(ctx, c.n, dtype)
    if phi is None:
        st.init_basis(0)
    else:
        st.from_numpy(phi.astype(np.complex128 if dtype == q.QSV_C128 else np.complex64))
    st.apply_circuit(c.gates, params=c.params if params is None else params, flags=flags)
    out = st.to_numpy()
    st.free()
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_jit_circuits_vs_oracle(q, dtype):
    dt = q.QSV_C128 if dtype == "c128" else q.QSV_C64
    ctx = q.Context()
    ctx.set_jit(1)
    cases = [W.layered_cnot_brick(16, 4, seed=801), W.layered_haar_pairs(15, 3, seed=802),
             W.random_mix(14, 120, seed=803), W.qft(13), W.random_multicontrol(14, 60, seed=804)]
    for c in cases:
        phi = W.random_state(c.n, 810)
        ref = O.run(c, phi)
        got = run(q, ctx, c, dt, phi)
        if dt == q.QSV_C128:
            assert np.max(np.abs(got - ref)) <= TOL128, c.name
        else:
            assert infidelity(got, ref) <= 1e-6, c.name
    kernels, secs = ctx.jit_stats()
    assert kernels > 0
    ctx.close()


@pytest.mark.parametrize("tb,rb,rounds", [(10, 2, 1), (11, 3, 2), (12, 3, 1), (12, 4, 2), (13, 4, 2),
                                          (13, 5, 1)])
def test_jit_every_tile_shape(q, tb, rb, rounds):
    ctx = q.Context()
    ctx.set_jit(1)
    ctx.set_tile(q.QSV_C128, tb, 0, rb, rounds)
    c = W.random_mix(15, 150, seed=820 + tb + rb)
    phi = W.random_state(15, 821)
    got = run(q, ctx, c, q.QSV_C128, phi)
    assert np.max(np.abs(got - O.run(c, phi))) <= TOL128
    ctx.close()


def test_jit_from_zero_new_angles_and_interpreter_agree(q):
    """FROM_ZERO on the first pass; new angles on the same structure reuse
    every kernel (no new compiles); the interpreting kernel gives the same
    amplitudes bit for bit (same register bodies, same order)."""
    c = W.hea_cz_ring(16, 4, seed=830)
    ctx = q.Context()
    ctx.set_jit(1)
    st = q.State(ctx, c.n, q.QSV_C128)
    st.apply_circuit(c.gates, params=c.params, flags=q.FLAG_FROM_ZERO)
    a = st.to_numpy()
    ref = O.run(c, np.eye(1, 2 ** c.n, 0, dtype=complex).ravel())
    assert np.max(np.abs(a - ref)) <= TOL128
    k1, _ = ctx.jit_stats()
    p2 = np.random.default_rng(831).uniform(0, 2 * np.pi, c.params.size)
    st.apply_circuit(c.gates, params=p2, flags=q.FLAG_FROM_ZERO)
    b = st.to_numpy()
    k2, _ = ctx.jit_stats()
    assert k2 == k1
    ref2 = O.run(W.Circuit(c.n, c.gates, p2), np.eye(1, 2 ** c.n, 0, dtype=complex).ravel())
    assert np.max(np.abs(b - ref2)) <= TOL128
    ctx.set_jit(0)
    st.apply_circuit(c.gates, params=p2, flags=q.FLAG_FROM_ZERO)
    assert np.array_equal(st.to_numpy(), b)
    st.free()
    ctx.close()


def test_jit_bench_circuit_equals_interpreter_at_30_qubits(q):
    """The benchmark's 30-qubit brick circuit in its launch configuration:
    the specialised pass kernels give the interpreting kernel's amplitudes
    bit for bit (the interpreting path is checked against the oracle at 28
    qubits)."""
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < 40 * 2 ** 30:
        pytest.skip("needs ~40 GiB of device memory")
    c = W.layered_cnot_brick(30, 20, seed=3002)
    ctx = q.Context()
    a = q.State(ctx, 30, q.QSV_C128)
    a.apply_circuit(c.gates, flags=q.FLAG_FROM_ZERO)
    ctx.set_jit(1)
    b = q.State(ctx, 30, q.QSV_C128)
    b.apply_circuit(c.gates, flags=q.FLAG_FROM_ZERO)
    assert torch.equal(a.tensor, b.tensor)
    a.free()
    b.free()
    ctx.close()


def test_jit_disk_cache(q, tmp_path, monkeypatch):
    """With QSV_JIT_CACHE set, a second context loads the kernels the first
    one compiled (no compile time) and gives the same amplitudes."""
    monkeypatch.setenv("QSV_JIT_CACHE", str(tmp_path))
    c = W.layered_haar_pairs(14, 3, seed=840)
    outs = []
    for k in range(2):
        ctx = q.Context()
        ctx.set_jit(1)
        outs.append(run(q, ctx, c, q.QSV_C128))
        kernels, secs = ctx.jit_stats()
        assert kernels > 0
        if k == 1:
            assert secs < 1.0
        ctx.close()
    assert np.array_equal(outs[0], outs[1])
    assert len(list(tmp_path.glob("qsv_pass_c128_*.co"))) > 0
